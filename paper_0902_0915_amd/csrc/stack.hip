// Kernel-stack gridding and degridding: each visibility selects one complex kernel (for
// instance a direction-dependent beam term combined with a w term) of its own support S,
// tabulated at O x O phases. Gridding adds K[py][px][s][t] * w * g1 * conj(g2) * V into the
// S x S footprint; degridding is the adjoint with conjugated taps.
//
// With supports up to 63 cells and sparse visibilities, a haloed scatter tile would be
// mostly halo, so the gridder gathers by output tile instead: every tile has a candidate
// list of the visibilities whose footprint touches it (built at plan time; a visibility
// appears in every tile its footprint overlaps), one wavefront owns one tile (or one band
// of its rows) as a private LDS accumulator, and the finished tile is stored to HBM
// exactly once. No atomics are needed anywhere. This is the gather form the paper's port
// used in place of scatter (Section 3.2), applied per tile rather than per grid cell.
#include "internal.h"

#include <algorithm>
#include <cstring>

namespace mwg {

Status sort_pairs(uint32_t *keys, uint32_t *keys_alt, const uint32_t *vals_init, uint32_t *vals,
                  uint32_t *vals_alt, int64_t n, int keybits, uint32_t **keys_out,
                  uint32_t **vals_out, hipStream_t s);
Status exclusive_scan_u32(uint32_t *data, int64_t n, hipStream_t s);
Status launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);

namespace {

constexpr int kBlock = 256;

unsigned grid1d(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

int bitlen(uint64_t v) {
    int r = 0;
    while (v) {
        r++;
        v >>= 1;
    }
    return r;
}


// Footprint tile span of a kept group: tiles [x0, x1] x [y0, y1].
__device__ inline void span(uint32_t p, int h, int T, int &x0, int &x1, int &y0, int &y1) {
    const int cx = (int)(p & 0xFFFu), cy = (int)((p >> 12) & 0xFFFu);
    x0 = (cx - h) / T;
    x1 = (cx + h) / T;
    y0 = (cy - h) / T;
    y1 = (cy + h) / T;
}

__global__ void k_pair_count(const uint32_t *pos, const int32_t *kidx, const int32_t *ksup,
                             int64_t ng, int T, uint32_t *count) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ng) return;
    const uint32_t p = pos[g];
    uint32_t n = 0;
    if (p != kDropped) {
        int x0, x1, y0, y1;
        span(p, (ksup[kidx[g]] - 1) / 2, T, x0, x1, y0, y1);
        n = (uint32_t)((x1 - x0 + 1) * (y1 - y0 + 1));
    }
    count[g] = n;
}

// Pair keys: tile, then (kernel, phase) so that consecutive candidates share a kernel slice.
__global__ void k_pair_emit(const uint32_t *pos, const int32_t *kidx, const int32_t *ksup,
                            int64_t ng, int T, int ntx, const uint32_t *offset, int sbits,
                            uint32_t *keys, uint32_t *vals) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ng) return;
    const uint32_t p = pos[g];
    if (p == kDropped) return;
    int x0, x1, y0, y1;
    const int k = kidx[g];
    span(p, (ksup[k] - 1) / 2, T, x0, x1, y0, y1);
    const uint32_t sec = sbits ? (((uint32_t)k << 8) | (p >> 24)) : 0u;
    uint32_t o = offset[g];
    for (int ty = y0; ty <= y1; ty++)
        for (int tx = x0; tx <= x1; tx++) {
            keys[o] = ((uint32_t)(ty * ntx + tx) << sbits) | sec;
            vals[o] = (uint32_t)g;
            o++;
        }
}

__global__ void k_pair_bounds(const uint32_t *skeys, int64_t n, int sbits, int32_t *tstart,
                              int32_t *tend) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t t = skeys[i] >> sbits;
    if (i == 0 || (skeys[i - 1] >> sbits) != t) tstart[t] = (int32_t)i;
    if (i == n - 1 || (skeys[i + 1] >> sbits) != t) tend[t] = (int32_t)(i + 1);
}

struct StackArgs {
    const float2 *vis, *gains, *kstack;
    const uint32_t *pos, *pairs, *ants;
    const int32_t *kidx, *ksup;
    const int64_t *koff;
    const float *w;
    const WorkItem *work;
    float2 *grid;
    int nx, ny, T, ntx, O, nchan, accumulate;
};

__device__ inline float rl_f(float x, int j) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), j));
}

// Row rounds of a candidate's clipped footprint whose tap loads are issued together (4 was
// measured faster than 2, 8, 16 or 24 on the beam x w-plane workload).
constexpr int kStackRounds = 4;

// A candidate of the stack gridder, set up and with the tap loads of its first chunk issued.
template <int NPOL>
struct Cand {
    int ya, yb, rpi, rl, o0, rowoff, S;  // rows [ya, yb]; tap row of grid row y: y + rowoff
    bool on;                             // this lane covers a footprint column
    const float2 *kb;                    // this lane's tap column
    float2 v[NPOL];                      // the candidate's weighted visibilities
    float2 K[kStackRounds];              // taps of the first chunk
};

// Row-round chunk at y0 of candidate c with taps K: the LDS read-add-writes.
template <int NPOL>
__device__ inline void stack_rmw(const Cand<NPOL> &c, int y0, const float2 (&K)[kStackRounds], float2 *tile, int T,
                                 int ty0) {
#pragma unroll
    for (int it = 0; it < kStackRounds; it++) {
        const int yy = y0 + it * c.rpi + c.rl;
        if (c.on && yy <= c.yb) {
            const int o = (yy - ty0) * T + c.o0;
#pragma unroll
            for (int q = 0; q < NPOL; q++) {
                float2 acc = tile[q * T * T + o];
                acc.x += K[it].x * c.v[q].x - K[it].y * c.v[q].y;
                acc.y += K[it].x * c.v[q].y + K[it].y * c.v[q].x;
                tile[q * T * T + o] = acc;
            }
        }
    }
}

// Tap loads of the chunk at y0, issued by every lane without a branch (a branch around each
// load would make the compiler wait for all loads in flight before the first use): a lane
// outside the footprint reads the tap of the footprint's last row in its column, an address
// in a line the active lanes fetch anyway, and keeps zero.
template <int NPOL>
__device__ inline void stack_load(const Cand<NPOL> &c, int y0, float2 (&K)[kStackRounds]) {
#pragma unroll
    for (int it = 0; it < kStackRounds; it++) {
        const int yy = y0 + it * c.rpi + c.rl;
        const float2 k = c.kb[(int64_t)(min(yy, c.yb) + c.rowoff) * c.S];
        K[it] = (c.on && yy <= c.yb) ? k : make_float2(0.f, 0.f);
    }
}

// Takes the next staged candidate of `todo` (its footprint meets the band), sets it up and
// issues its first chunk's tap loads; with `todo` empty, a dummy whose lanes are all off.
template <int NPOL>
__device__ inline void stack_prep(const StackArgs &a, uint64_t &todo, uint32_t qp, int qS, int64_t qoff,
                                  const float2 (&qv)[NPOL], int lane, int tab_rows, int tab_mul, int tx0, int ylo,
                                  int yhi, int T, Cand<NPOL> &c) {
    const bool real = todo != 0;
    const int j = real ? (int)__builtin_ctzll(todo) : 0;
    todo = real ? todo & (todo - 1) : 0;
    const uint32_t p = (uint32_t)__builtin_amdgcn_readlane((int)qp, j);
    const int S = __builtin_amdgcn_readlane(qS, j);
    const uint32_t olo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)qoff, j);
    const uint32_t ohi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)qoff >> 32), j);
    const int64_t koff = (int64_t)(((uint64_t)ohi << 32) | olo);
    const int h = (S - 1) / 2;
    const int cx = (int)(p & 0xFFFu), cy = (int)((p >> 12) & 0xFFFu);
    const int px = (int)((p >> 24) & 0xFu), py = (int)(p >> 28);
    c.ya = max(cy - h, ylo);
    c.yb = real ? min(cy + h, yhi) : c.ya - 1;
    const int xa = max(cx - h, tx0), xb = real ? min(cx + h, tx0 + T - 1) : xa;
#pragma unroll
    for (int q = 0; q < NPOL; q++) c.v[q] = make_float2(rl_f(qv[q].x, j), rl_f(qv[q].y, j));
    const int ncol = xb - xa + 1;
    c.rpi = __builtin_amdgcn_readlane(tab_rows, ncol - 1);
    c.rl = (lane * __builtin_amdgcn_readlane(tab_mul, ncol - 1)) >> 16;
    const int cl = lane - c.rl * ncol;
    c.on = real && c.rl < c.rpi;
    c.S = S;
    c.rowoff = h - cy;
    c.kb = a.kstack + koff + ((int64_t)(py * a.O + px) * S) * S + (cl + xa - cx + h);
    c.o0 = xa + cl - tx0;
    stack_load<NPOL>(c, c.ya, c.K);
}

// The LDS work of a prepared candidate: its first chunk, then the others chunk by chunk.
template <int NPOL>
__device__ inline void stack_finish(const Cand<NPOL> &c, float2 *tile, int T, int ty0) {
    stack_rmw<NPOL>(c, c.ya, c.K, tile, T, ty0);
    for (int y0 = c.ya + kStackRounds * c.rpi; y0 <= c.yb; y0 += kStackRounds * c.rpi) {
        float2 K[kStackRounds];
        stack_load<NPOL>(c, y0, K);
        stack_rmw<NPOL>(c, y0, K, tile, T, ty0);
    }
}

// One wavefront per work item (tile, candidate range, row band); private LDS tile. At most 8
// waves per workgroup (the plan refuses more).
template <int NPOL>
__global__ __launch_bounds__(512) void k_grid_stack(StackArgs a, int nwork) {
    extern __shared__ __align__(16) float smem[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nwaves = blockDim.x >> 6;
    const int widx = blockIdx.x * nwaves + wave;
    if (widx >= nwork) return;
    const int T = a.T;
    float2 *tile = (float2 *)smem + (size_t)wave * NPOL * T * T;
    // Per clipped footprint width n = lane + 1 (1 ... 64; tiles are at most 64 wide): the rows
    // one round of 64 lanes covers (64 / n) and the multiplier m = ceil(2^16 / n) with
    // j / n = (j * m) >> 16 for every j < 64. A candidate picks its width's entries with
    // v_readlane, so that it needs neither an integer division nor a memory load.
    const int tab_rows = 64 / (lane + 1), tab_mul = (65536 + lane) / (lane + 1);
    const WorkItem wk = a.work[widx];
    const int r0 = wk.pad & 0xFFFF, r1 = wk.pad >> 16;
    const int tx0 = (wk.tile % a.ntx) * T, ty0 = (wk.tile / a.ntx) * T;
    const int ylo = ty0 + r0, yhi = ty0 + r1 - 1;
    for (int i = lane; i < NPOL * T * T; i += 64) tile[i] = make_float2(0.f, 0.f);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    for (int base = wk.begin; base < wk.end; base += 64) {
        const int cnt = min(64, wk.end - base);
        // lane j stages candidate j: position, kernel support and offset, multiplied
        // visibilities (all loads of the batch in flight together)
        uint32_t qp = kDropped;
        int qS = 1;
        int64_t qoff = 0;
        float2 qv[NPOL];
        for (int p = 0; p < NPOL; p++) qv[p] = make_float2(0.f, 0.f);
        if (lane < cnt) {
            const uint32_t g = a.pairs[base + lane];
            qp = a.pos[g];
            const int qk = a.kidx[g];
            qS = a.ksup[qk];
            qoff = a.koff[qk];
            float mr = a.w ? a.w[g] : 1.0f, mi = 0.0f;
            if (a.gains) {
                const uint32_t an = a.ants[(int64_t)g / a.nchan];
                const float2 g1 = a.gains[an & 0xFFFFu], g2 = a.gains[an >> 16];
                const float gr = g1.x * g2.x + g1.y * g2.y, gi = g1.y * g2.x - g1.x * g2.y;
                mi = mr * gi;
                mr = mr * gr;
            }
            for (int p = 0; p < NPOL; p++) {
                const float2 v = a.vis[(int64_t)g * NPOL + p];
                qv[p] = make_float2(mr * v.x - mi * v.y, mr * v.y + mi * v.x);
            }
        }
        // candidates whose clipped footprint meets this item's band of rows
        uint64_t todo;
        {
            const int hS = (qS - 1) / 2;
            const int cxl = (int)(qp & 0xFFFu), cyl = (int)((qp >> 12) & 0xFFFu);
            const bool meets = lane < cnt && max(cyl - hS, ylo) <= min(cyl + hS, yhi) &&
                               max(cxl - hS, tx0) <= min(cxl + hS, tx0 + T - 1);
            todo = __ballot(meets);
        }
        // Candidates in pairs: both are set up and both first chunks' tap loads issued, in
        // straight-line code (a missing second candidate is a dummy whose lanes are all off),
        // before the LDS work of either, so that the two load latencies overlap.
        while (todo) {
            Cand<NPOL> A, B;
            stack_prep<NPOL>(a, todo, qp, qS, qoff, qv, lane, tab_rows, tab_mul, tx0, ylo, yhi, T, A);
            stack_prep<NPOL>(a, todo, qp, qS, qoff, qv, lane, tab_rows, tab_mul, tx0, ylo, yhi, T, B);
            stack_finish<NPOL>(A, tile, T, ty0);
            stack_finish<NPOL>(B, tile, T, ty0);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int q = 0; q < NPOL; q++)
        for (int i = lane; i < (r1 - r0) * T; i += 64) {
            const int r = r0 + i / T, c = i % T;
            const int gy = ty0 + r, gx = tx0 + c;
            if (gy >= a.ny || gx >= a.nx) continue;
            float2 *dst = a.grid + ((int64_t)q * a.ny + gy) * a.nx + gx;
            float2 v = tile[q * T * T + r * T + c];
            if (a.accumulate) {
                const float2 o = *dst;
                v.x += o.x;
                v.y += o.y;
            }
            *dst = v;
        }
}

struct StackDegridArgs {
    const float2 *grid, *gains, *vis_in, *kstack;
    float2 *vis_out, *grad_gains;
    const uint32_t *perm, *spos, *sant, *skid;
    const int32_t *ksup;
    const int64_t *koff;
    const float *sw;
    int64_t nkept;
    int nx, ny, O;
};

// One wavefront per kept group: lanes over the S x S taps, conjugated, then a cross-lane
// reduction.
template <int NPOL>
__global__ __launch_bounds__(256) void k_degrid_stack(StackDegridArgs a) {
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (i >= a.nkept) return;
    const uint32_t p = a.spos[i];
    const int k = (int)a.skid[i];
    const int S = a.ksup[k], h = (S - 1) / 2;
    const int cx = (int)(p & 0xFFFu), cy = (int)((p >> 12) & 0xFFFu);
    const int px = (int)((p >> 24) & 0xFu), py = (int)(p >> 28);
    const float2 *kb = a.kstack + a.koff[k] + ((int64_t)(py * a.O + px) * S) * S;
    float2 acc[NPOL];
#pragma unroll
    for (int q = 0; q < NPOL; q++) acc[q] = make_float2(0.f, 0.f);
    for (int idx = lane; idx < S * S; idx += 64) {
        const int s = idx / S, t = idx - s * S;
        const float2 K = kb[idx];
        const int64_t cell = (int64_t)(cy - h + s) * a.nx + (cx - h + t);
#pragma unroll
        for (int q = 0; q < NPOL; q++) {
            const float2 G = a.grid[(int64_t)q * a.nx * a.ny + cell];
            acc[q].x += K.x * G.x + K.y * G.y; // conj(K) * G
            acc[q].y += K.x * G.y - K.y * G.x;
        }
    }
#pragma unroll
    for (int q = 0; q < NPOL; q++)
        for (int o = 32; o > 0; o >>= 1) {
            acc[q].x += __shfl_xor(acc[q].x, o, 64);
            acc[q].y += __shfl_xor(acc[q].y, o, 64);
        }
    if (lane != 0) return;
    const float w = a.sw ? a.sw[i] : 1.0f;
    const uint32_t gi = a.perm[i];
    float2 y[NPOL], out[NPOL];
#pragma unroll
    for (int q = 0; q < NPOL; q++) {
        y[q] = make_float2(w * acc[q].x, w * acc[q].y);
        out[q] = y[q];
    }
    if (a.gains) {
        const uint32_t an = a.sant[i];
        const int a1 = (int)(an & 0xFFFFu), a2 = (int)(an >> 16);
        const float2 g1 = a.gains[a1], g2 = a.gains[a2];
        const float mr = g1.x * g2.x + g1.y * g2.y, mi = g1.x * g2.y - g1.y * g2.x;
#pragma unroll
        for (int q = 0; q < NPOL; q++)
            out[q] = make_float2(mr * y[q].x - mi * y[q].y, mr * y[q].y + mi * y[q].x);
        if (a.grad_gains) {
            float2 t1 = make_float2(0.f, 0.f);
#pragma unroll
            for (int q = 0; q < NPOL; q++) {
                const float2 V = a.vis_in[(int64_t)gi * NPOL + q];
                t1.x += V.x * y[q].x + V.y * y[q].y;
                t1.y += V.x * y[q].y - V.y * y[q].x;
            }
            const float2 t2 = make_float2(t1.x, -t1.y);
            atomicAdd(&a.grad_gains[a1].x, g2.x * t1.x - g2.y * t1.y);
            atomicAdd(&a.grad_gains[a1].y, g2.x * t1.y + g2.y * t1.x);
            atomicAdd(&a.grad_gains[a2].x, g1.x * t2.x - g1.y * t2.y);
            atomicAdd(&a.grad_gains[a2].y, g1.x * t2.y + g1.y * t2.x);
        }
    }
#pragma unroll
    for (int q = 0; q < NPOL; q++) a.vis_out[(int64_t)gi * NPOL + q] = out[q];
}

template <int NPOL>
__global__ void k_zero_dropped_stack(float2 *vis_out, const uint32_t *dropped, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
#pragma unroll
    for (int q = 0; q < NPOL; q++) vis_out[(int64_t)dropped[i] * NPOL + q] = make_float2(0.f, 0.f);
}

template <int NPOL>
Status grid_stack_npol(Instance &I, StackArgs &a, hipStream_t s) {
    const int nw = I.L.wg_waves;
    const size_t lds = sizeof(float2) * (size_t)nw * NPOL * a.T * a.T;
    if (lds > 160 * 1024) return make_error(MW_ERR_UNSUPPORTED, "stack tile needs %zu B of LDS", lds);
    if (I.nwork > 0) {
        hipLaunchKernelGGL(k_grid_stack<NPOL>, dim3((I.nwork + nw - 1) / nw), dim3(64 * nw), lds, s, a,
                           I.nwork);
        MWG_HIP(hipGetLastError());
    }
    return Status::Ok();
}

template <int NPOL>
Status degrid_stack_npol(Instance &I, StackDegridArgs &a, hipStream_t s) {
    const int64_t ndropped = I.ngroups - I.nkept;
    if (ndropped > 0) {
        hipLaunchKernelGGL(k_zero_dropped_stack<NPOL>, dim3(grid1d(ndropped)), dim3(kBlock), 0, s,
                           a.vis_out, (const uint32_t *)I.dropped, ndropped);
        MWG_HIP(hipGetLastError());
    }
    if (I.nkept > 0) {
        hipLaunchKernelGGL(k_degrid_stack<NPOL>, dim3((unsigned)((I.nkept + 3) / 4)), dim3(256), 0, s, a);
        MWG_HIP(hipGetLastError());
    }
    return Status::Ok();
}

} // namespace

size_t stack_lds(int npol, int T, int waves) { return sizeof(float2) * (size_t)waves * npol * T * T; }

// Candidate pairs, sorted by (tile, kernel, phase); one work item per tile or row band.
Status build_stack_schedule(Instance &I, const Launch &L, hipStream_t s) {
    const int64_t ng = I.ngroups;
    const int T = L.tile;
    const int ntx = (I.nx + T - 1) / T, nty = (I.ny + T - 1) / T;
    const int64_t ntiles = (int64_t)ntx * nty;
    I.L = L;
    I.ntx = ntx;
    I.nty = nty;
    DevTmp counts;
    MWG_TRY(counts.alloc(4 * (size_t)(ng + 1), s));
    MWG_TRY(launch_fill_u32(counts.as<uint32_t>(), ng + 1, 0, s));
    if (ng > 0) {
        hipLaunchKernelGGL(k_pair_count, dim3(grid1d(ng)), dim3(kBlock), 0, s, I.pos, I.kidx_orig, I.ksup,
                           ng, T, counts.as<uint32_t>());
        MWG_HIP(hipGetLastError());
    }
    MWG_TRY(exclusive_scan_u32(counts.as<uint32_t>(), ng + 1, s));
    uint32_t npairs = 0;
    MWG_HIP(hipMemcpyAsync(&npairs, counts.as<uint32_t>() + ng, 4, hipMemcpyDeviceToHost, s));
    MWG_HIP(hipStreamSynchronize(s));
    const int tbits = bitlen((uint64_t)ntiles);
    const int kbits = bitlen((uint64_t)std::max(I.nkernel - 1, 1));
    const int sbits = (tbits + kbits + 8 <= 32) ? kbits + 8 : 0;
    void *p;
    std::vector<WorkItem> items;
    int nonempty = 0;
    if (npairs > 0) {
        DevTmp keys, keys2, vals, vals2, vinit;
        MWG_TRY(keys.alloc(4 * (size_t)npairs, s));
        MWG_TRY(keys2.alloc(4 * (size_t)npairs, s));
        MWG_TRY(vals.alloc(4 * (size_t)npairs, s));
        MWG_TRY(vals2.alloc(4 * (size_t)npairs, s));
        MWG_TRY(vinit.alloc(4 * (size_t)npairs, s));
        hipLaunchKernelGGL(k_pair_emit, dim3(grid1d(ng)), dim3(kBlock), 0, s, I.pos, I.kidx_orig, I.ksup, ng,
                           T, ntx, counts.as<uint32_t>(), sbits, keys.as<uint32_t>(), vinit.as<uint32_t>());
        MWG_HIP(hipGetLastError());
        uint32_t *sk = nullptr, *sv = nullptr;
        MWG_TRY(sort_pairs(keys.as<uint32_t>(), keys2.as<uint32_t>(), vinit.as<uint32_t>(),
                           vals.as<uint32_t>(), vals2.as<uint32_t>(), npairs, tbits + sbits, &sk, &sv, s));
        MWG_TRY(I.arena.alloc(&p, 4 * (size_t)npairs));
        I.pairs = (uint32_t *)p;
        I.npairs = npairs;
        MWG_HIP(hipMemcpyAsync(I.pairs, sv, 4 * (size_t)npairs, hipMemcpyDeviceToDevice, s));
        DevTmp tstart, tend;
        MWG_TRY(tstart.alloc(4 * ntiles, s));
        MWG_TRY(tend.alloc(4 * ntiles, s));
        MWG_TRY(launch_fill_u32(tstart.as<uint32_t>(), ntiles, 0, s));
        MWG_TRY(launch_fill_u32(tend.as<uint32_t>(), ntiles, 0, s));
        hipLaunchKernelGGL(k_pair_bounds, dim3(grid1d(npairs)), dim3(kBlock), 0, s, sk, (int64_t)npairs, sbits,
                           tstart.as<int32_t>(), tend.as<int32_t>());
        MWG_HIP(hipGetLastError());
        std::vector<int32_t> hs(ntiles), he(ntiles);
        MWG_HIP(hipMemcpyAsync(hs.data(), tstart.p, 4 * ntiles, hipMemcpyDeviceToHost, s));
        MWG_HIP(hipMemcpyAsync(he.data(), tend.p, 4 * ntiles, hipMemcpyDeviceToHost, s));
        MWG_HIP(hipStreamSynchronize(s));
        for (int64_t t = 0; t < ntiles; t++) {
            const int cnt = he[t] - hs[t];
            if (cnt <= 0) continue;
            nonempty++;
            // heavy tiles are split into bands of rows, each a work item of its own
            int bands = std::min(T, std::max(1, (cnt + L.split - 1) / L.split));
            for (int b = 0; b < bands; b++) {
                WorkItem w;
                w.tile = (int32_t)t;
                w.begin = hs[t];
                w.end = he[t];
                const int r0 = T * b / bands, r1 = T * (b + 1) / bands;
                w.pad = r0 | (r1 << 16);
                items.push_back(w);
            }
        }
        std::stable_sort(items.begin(), items.end(), [](const WorkItem &x, const WorkItem &y) {
            return (int64_t)(x.end - x.begin) * ((x.pad >> 16) - (x.pad & 0xFFFF)) >
                   (int64_t)(y.end - y.begin) * ((y.pad >> 16) - (y.pad & 0xFFFF));
        });
    }
    I.ntiles_nonempty = nonempty;
    I.nwork = (int)items.size();
    MWG_TRY(I.arena.alloc(&p, sizeof(WorkItem) * std::max<size_t>(items.size(), 1)));
    I.work = (WorkItem *)p;
    if (!items.empty())
        MWG_HIP(hipMemcpyAsync(I.work, items.data(), sizeof(WorkItem) * items.size(), hipMemcpyHostToDevice, s));
    MWG_HIP(hipStreamSynchronize(s));
    return Status::Ok();
}

Status launch_grid_stack(Instance &I, const float2 *vis, const float2 *gains, float2 *grid, int accumulate,
                         hipStream_t s) {
    if (!accumulate) MWG_TRY(launch_fill_zero(grid, sizeof(float2) * (size_t)I.npol * I.nx * I.ny, s));
    StackArgs a{};
    a.vis = vis;
    a.gains = gains;
    a.kstack = I.kstack;
    a.pos = I.pos;
    a.pairs = I.pairs;
    a.ants = I.ant_orig;
    a.kidx = I.kidx_orig;
    a.ksup = I.ksup;
    a.koff = I.koff;
    a.w = I.w_orig;
    a.work = I.work;
    a.grid = grid;
    a.nx = I.nx;
    a.ny = I.ny;
    a.T = I.L.tile;
    a.ntx = I.ntx;
    a.O = I.O;
    a.nchan = I.nchan;
    a.accumulate = 1; // the grid was zeroed above in overwrite mode
    switch (I.npol) {
    case 1: return grid_stack_npol<1>(I, a, s);
    case 2: return grid_stack_npol<2>(I, a, s);
    case 4: return grid_stack_npol<4>(I, a, s);
    default: return make_error(MW_ERR_UNSUPPORTED, "npol %d", I.npol);
    }
}

Status launch_degrid_stack(Instance &I, const float2 *grid, const float2 *gains, const float2 *vis_in,
                           float2 *vis_out, float2 *grad_gains, hipStream_t s) {
    if (grad_gains) MWG_TRY(launch_fill_zero(grad_gains, sizeof(float2) * (size_t)I.nant, s));
    StackDegridArgs a{};
    a.grid = grid;
    a.gains = gains;
    a.vis_in = vis_in;
    a.kstack = I.kstack;
    a.vis_out = vis_out;
    a.grad_gains = grad_gains;
    a.perm = I.perm;
    a.spos = I.spos;
    a.sant = I.sant;
    a.skid = I.skid;
    a.ksup = I.ksup;
    a.koff = I.koff;
    a.sw = I.sw;
    a.nkept = I.nkept;
    a.nx = I.nx;
    a.ny = I.ny;
    a.O = I.O;
    switch (I.npol) {
    case 1: return degrid_stack_npol<1>(I, a, s);
    case 2: return degrid_stack_npol<2>(I, a, s);
    case 4: return degrid_stack_npol<4>(I, a, s);
    default: return make_error(MW_ERR_UNSUPPORTED, "npol %d", I.npol);
    }
}

} // namespace mwg
