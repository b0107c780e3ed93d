// Shared device code of the separable degridder, used by the single-instance kernel
// (degrid.hip) and the batched kernel (batched.hip).
#pragma once

#include "internal.h"

namespace mwg {

struct DegridArgs {
    const float2 *grid, *gains, *vis_in;
    float2 *vis_out, *grad_gains;
    const uint32_t *perm, *spos, *sant;
    const float *sw;
    const WorkItem *work;
    const float *tab;
    int nx, ny, T, ntx, W, O, nant, ant_in_lds;
};

// Threads per degridder workgroup for work items of (on average) groups_per_item groups: one
// thread per group, 64 to 256, so that sparse plans do not leave most of each workgroup idle.
inline int degrid_threads(int64_t groups, int64_t items) {
    const int64_t avg = items > 0 ? groups / items : 0;
    return avg <= 64 ? 64 : (avg <= 128 ? 128 : 256);
}

// A group's footprint sum y[p] = sum_s T[py][s] sum_t T[px][t] G[p][row s][col t] from the
// LDS tile g (row stride R, planes of R * R) at offset o: each row's sum over t first, then
// the row tap. With the support a compile-time WT the column taps stay in registers and the
// window loads pair up; WT = 0 takes the support at run time (any W <= 15).
template <int NPOL, int WT>
__device__ inline void degrid_footprint(const float2 *g, const float *tab, int R, int Wrt, int o, int px, int py,
                                        float2 (&acc)[NPOL]) {
#pragma unroll
    for (int p = 0; p < NPOL; p++) acc[p] = make_float2(0.f, 0.f);
    if constexpr (WT > 0) {
        float tx[WT];
#pragma unroll
        for (int t = 0; t < WT; t++) tx[t] = tab[px * WT + t];
        // rows one at a time (unrolling them too hoists every window load and spills)
#pragma unroll 1
        for (int sy = 0; sy < WT; sy++) {
            const float ty = tab[py * WT + sy];
            const float2 *row = g + o + sy * R;
            float2 rs[NPOL];
#pragma unroll
            for (int p = 0; p < NPOL; p++) rs[p] = make_float2(0.f, 0.f);
#pragma unroll
            for (int sx = 0; sx < WT; sx++) {
#pragma unroll
                for (int p = 0; p < NPOL; p++) {
                    const float2 v = row[(size_t)p * R * R + sx];
                    rs[p].x = fmaf(tx[sx], v.x, rs[p].x);
                    rs[p].y = fmaf(tx[sx], v.y, rs[p].y);
                }
            }
#pragma unroll
            for (int p = 0; p < NPOL; p++) {
                acc[p].x = fmaf(ty, rs[p].x, acc[p].x);
                acc[p].y = fmaf(ty, rs[p].y, acc[p].y);
            }
        }
    } else {
        for (int sy = 0; sy < Wrt; sy++) {
            const float ty = tab[py * Wrt + sy];
            const float2 *row = g + o + sy * R;
            float2 rs[NPOL];
#pragma unroll
            for (int p = 0; p < NPOL; p++) rs[p] = make_float2(0.f, 0.f);
            for (int sx = 0; sx < Wrt; sx++) {
                const float tx = tab[px * Wrt + sx];
#pragma unroll
                for (int p = 0; p < NPOL; p++) {
                    const float2 v = row[(size_t)p * R * R + sx];
                    rs[p].x = fmaf(tx, v.x, rs[p].x);
                    rs[p].y = fmaf(tx, v.y, rs[p].y);
                }
            }
#pragma unroll
            for (int p = 0; p < NPOL; p++) {
                acc[p].x = fmaf(ty, rs[p].x, acc[p].x);
                acc[p].y = fmaf(ty, rs[p].y, acc[p].y);
            }
        }
    }
}

// NPOL complex values of one group's record (16-byte aligned for NPOL >= 2) in one or two
// vector accesses.
template <int NPOL>
__device__ inline void load_record(const float2 *src, float2 (&v)[NPOL]) {
    if constexpr (NPOL == 4) {
        const float4 x = ((const float4 *)src)[0], y = ((const float4 *)src)[1];
        v[0] = make_float2(x.x, x.y);
        v[1] = make_float2(x.z, x.w);
        v[2] = make_float2(y.x, y.y);
        v[3] = make_float2(y.z, y.w);
    } else if constexpr (NPOL == 2) {
        const float4 x = ((const float4 *)src)[0];
        v[0] = make_float2(x.x, x.y);
        v[1] = make_float2(x.z, x.w);
    } else {
        v[0] = src[0];
    }
}
template <int NPOL>
__device__ inline void store_record(float2 *dst, const float2 (&v)[NPOL]) {
    if constexpr (NPOL == 4) {
        ((float4 *)dst)[0] = make_float4(v[0].x, v[0].y, v[1].x, v[1].y);
        ((float4 *)dst)[1] = make_float4(v[2].x, v[2].y, v[3].x, v[3].y);
    } else if constexpr (NPOL == 2) {
        ((float4 *)dst)[0] = make_float4(v[0].x, v[0].y, v[1].x, v[1].y);
    } else {
        dst[0] = v[0];
    }
}

// The end of one group's degrid: weight, the gain product conj(g1) g2, the gains' gradient
// sums (into LDS when gacc holds them, else HBM) and the store of the record.
template <int NPOL>
__device__ inline void degrid_finish(const DegridArgs &a, int64_t i, float2 (&acc)[NPOL], bool want_g, float2 *gacc) {
    const float w = a.sw ? a.sw[i] : 1.0f;
#pragma unroll
    for (int p = 0; p < NPOL; p++) {
        acc[p].x *= w;
        acc[p].y *= w;
    }
    const uint32_t gi = a.perm[i];
    float2 out[NPOL];
    if (a.gains) {
        const uint32_t an = a.sant[i];
        const int a1 = (int)(an & 0xFFFFu), a2 = (int)(an >> 16);
        const float2 g1 = a.gains[a1], g2 = a.gains[a2];
        // conj(g1) * g2
        const float mr = g1.x * g2.x + g1.y * g2.y, mi = g1.x * g2.y - g1.y * g2.x;
#pragma unroll
        for (int p = 0; p < NPOL; p++)
            out[p] = make_float2(mr * acc[p].x - mi * acc[p].y, mr * acc[p].y + mi * acc[p].x);
        if (want_g) {
            float2 t1 = make_float2(0.f, 0.f), t2 = make_float2(0.f, 0.f);
            float2 vin[NPOL];
            load_record<NPOL>(a.vis_in + (int64_t)gi * NPOL, vin);
#pragma unroll
            for (int p = 0; p < NPOL; p++) {
                const float2 V = vin[p], y = acc[p];
                // conj(V) * y and V * conj(y)
                const float cr = V.x * y.x + V.y * y.y, ci = V.x * y.y - V.y * y.x;
                t1.x += cr;
                t1.y += ci;
                t2.x += cr;
                t2.y -= ci;
            }
            // grad[a1] += g2 * t1 ; grad[a2] += g1 * t2
            const float2 d1 = make_float2(g2.x * t1.x - g2.y * t1.y, g2.x * t1.y + g2.y * t1.x);
            const float2 d2 = make_float2(g1.x * t2.x - g1.y * t2.y, g1.x * t2.y + g1.y * t2.x);
            float2 *dst = a.ant_in_lds ? gacc : a.grad_gains;
            atomicAdd(&dst[a1].x, d1.x);
            atomicAdd(&dst[a1].y, d1.y);
            atomicAdd(&dst[a2].x, d2.x);
            atomicAdd(&dst[a2].y, d2.y);
        }
    } else {
#pragma unroll
        for (int p = 0; p < NPOL; p++) out[p] = acc[p];
    }
    store_record<NPOL>(a.vis_out + (int64_t)gi * NPOL, out);
}

// One workgroup grids-back one work item: stage its haloed grid tile in LDS, then one
// thread per group gathers the footprint. smem is the workgroup's dynamic LDS. WT: the
// support as a compile-time constant (0: a.W at run time).
template <int NPOL, int WT>
__device__ inline void degrid_item(const DegridArgs &a, const WorkItem wk, float *smem) {
    const int nthreads = blockDim.x, tid = threadIdx.x;
    const int T = a.T, W = WT > 0 ? WT : a.W, h = (W - 1) / 2, R = T + W - 1;
    const int tx0 = (wk.tile % a.ntx) * T, ty0 = (wk.tile / a.ntx) * T;
    float2 *g = (float2 *)smem;                      // [NPOL][R][R]
    float *tab = (float *)(g + (size_t)NPOL * R * R); // [O][W]
    float2 *gacc = (float2 *)(tab + ((a.O * W + 1) & ~1)); // [nant] when in LDS
    for (int idx = tid; idx < NPOL * R * R; idx += nthreads) {
        const int p = idx / (R * R), rc = idx - p * R * R;
        const int r = rc / R, c = rc - r * R;
        const int gy = ty0 - h + r, gx = tx0 - h + c;
        float2 v = make_float2(0.f, 0.f);
        if (gy >= 0 && gy < a.ny && gx >= 0 && gx < a.nx) v = a.grid[((int64_t)p * a.ny + gy) * a.nx + gx];
        g[idx] = v;
    }
    for (int i = tid; i < a.O * W; i += nthreads) tab[i] = a.tab[i];
    const bool want_g = a.grad_gains != nullptr;
    if (want_g && a.ant_in_lds)
        for (int i = tid; i < a.nant; i += nthreads) gacc[i] = make_float2(0.f, 0.f);
    __syncthreads();
    for (int64_t i = wk.begin + tid; i < wk.end; i += nthreads) {
        const uint32_t pp = a.spos[i];
        const int cx = (int)(pp & 0xFFFu), cy = (int)((pp >> 12) & 0xFFFu);
        const int px = (int)((pp >> 24) & 0xFu), py = (int)(pp >> 28);
        const int o = (cy - ty0) * R + (cx - tx0);
        float2 acc[NPOL];
        degrid_footprint<NPOL, WT>(g, tab, R, W, o, px, py, acc);
        degrid_finish<NPOL>(a, i, acc, want_g, gacc);
    }
    if (want_g && a.ant_in_lds) {
        __syncthreads();
        for (int i = tid; i < a.nant; i += nthreads) {
            const float2 v = gacc[i];
            if (v.x != 0.0f) atomicAdd(&a.grad_gains[i].x, v.x);
            if (v.y != 0.0f) atomicAdd(&a.grad_gains[i].y, v.y);
        }
    }
}

// The degridder over (cell, py) runs, for a compile-time support W in {3, 5, 7}. The groups
// of a run share the row contraction R[t][p] = sum_s T[py][s] G[p][cy+s][cx+t], so that
// y[p] = sum_t T[px][t] R[t][p]: R is formed once per run (W x W x NPOL taps read from LDS)
// and each group then reads only its run's W x NPOL values, instead of every group reading
// its whole footprint. Each wave takes chunks of 64 consecutive sorted groups; a ballot marks
// where a run starts (the first group of the chunk, or a change of (cx, cy, py)); rounds of
// up to kDegridRuns runs compute their R (one lane per run and column t) into the wave's LDS
// slice, then every group of those runs contracts it with its column taps.
constexpr int kDegridRuns = 18;

// LDS bytes of the run degridder: tile, 8-padded tap rows, per-antenna sums, wave slices.
inline size_t degrid_runs_lds(int npol, int T, int W, int O, int nwaves, int nant_lds) {
    const int R = T + W - 1;
    return sizeof(float2) * (size_t)npol * R * R + 32 * (size_t)O + sizeof(float2) * (size_t)((nant_lds + 1) & ~1) +
           (size_t)nwaves * (256 + (size_t)kDegridRuns * W * npol * sizeof(float2));
}

template <int NPOL, int W>
__device__ inline void degrid_item_runs(const DegridArgs &a, const WorkItem wk, float *smem) {
    const int nthreads = blockDim.x, tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), nwaves = nthreads >> 6;
    const int T = a.T, h = (W - 1) / 2, R = T + W - 1, RR = R * R;
    const int tx0 = (wk.tile % a.ntx) * T, ty0 = (wk.tile / a.ntx) * T;
    float2 *g = (float2 *)smem;                                  // [NPOL][R][R]
    float *tab8 = (float *)(g + (size_t)NPOL * RR);              // [O][8], zero past W
    float2 *gacc = (float2 *)(tab8 + 8 * a.O);                   // [nant] when in LDS
    const int nant_lds = a.ant_in_lds ? ((a.nant + 1) & ~1) : 0;
    uint32_t *rinfo = (uint32_t *)(gacc + nant_lds) + wave * (64 + kDegridRuns * W * NPOL * 2);
    float2 *rbuf = (float2 *)(rinfo + 64);                       // [kDegridRuns][W][NPOL]
    for (int idx = tid; idx < NPOL * RR; idx += nthreads) {
        const int p = idx / RR, rc = idx - p * RR;
        const int r = rc / R, c = rc - r * R;
        const int gy = ty0 - h + r, gx = tx0 - h + c;
        float2 v = make_float2(0.f, 0.f);
        if (gy >= 0 && gy < a.ny && gx >= 0 && gx < a.nx) v = a.grid[((int64_t)p * a.ny + gy) * a.nx + gx];
        g[idx] = v;
    }
    for (int i = tid; i < 8 * a.O; i += nthreads) {
        const int row = i >> 3, s = i & 7;
        tab8[i] = s < W ? a.tab[row * W + s] : 0.0f;
    }
    const bool want_g = a.grad_gains != nullptr;
    if (want_g && a.ant_in_lds)
        for (int i = tid; i < a.nant; i += nthreads) gacc[i] = make_float2(0.f, 0.f);
    __syncthreads();
    for (int64_t c0 = wk.begin + 64 * (int64_t)wave; c0 < wk.end; c0 += 64 * (int64_t)nwaves) {
        const int64_t i = c0 + lane;
        const bool live = i < wk.end;
        const uint32_t pp = live ? a.spos[i] : 0u;
        const int cx = (int)(pp & 0xFFFu), cy = (int)((pp >> 12) & 0xFFFu);
        const int px = (int)((pp >> 24) & 0xFu), py = (int)(pp >> 28);
        const uint32_t key = pp & 0xF0FFFFFFu;  // (cx, cy, py)
        const uint32_t prev = (uint32_t)__shfl_up((int)key, 1, 64);
        const bool start = live && (lane == 0 || key != prev);
        const uint64_t smask = __ballot(start);
        const int nr = __popcll(smask);
        const int rid = __popcll(smask & ((2ull << lane) - 1ull)) - 1;  // run of this lane's group
        if (start) rinfo[rid] = (uint32_t)((cy - ty0) * R + (cx - tx0)) | ((uint32_t)py << 16);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        float2 y[NPOL];
#pragma unroll
        for (int p = 0; p < NPOL; p++) y[p] = make_float2(0.f, 0.f);
        for (int r0 = 0; r0 < nr; r0 += kDegridRuns) {
            const int nrr = min(kDegridRuns, nr - r0);
            // R of runs [r0, r0 + nrr): one lane per (run, column)
            for (int u = lane; u < nrr * W; u += 64) {
                const int r = u / W, t = u - r * W;
                const uint32_t inf = rinfo[r0 + r];
                const int o = (int)(inf & 0xFFFFu) + t, ty8 = (int)(inf >> 16) * 8;
                const float4 q0 = *(const float4 *)(tab8 + ty8), q1 = *(const float4 *)(tab8 + ty8 + 4);
                const float ty[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
                float2 acc[NPOL];
#pragma unroll
                for (int p = 0; p < NPOL; p++) acc[p] = make_float2(0.f, 0.f);
#pragma unroll
                for (int s = 0; s < W; s++) {
#pragma unroll
                    for (int p = 0; p < NPOL; p++) {
                        const float2 v = g[p * RR + o + s * R];
                        acc[p].x = fmaf(ty[s], v.x, acc[p].x);
                        acc[p].y = fmaf(ty[s], v.y, acc[p].y);
                    }
                }
                store_record<NPOL>(rbuf + (size_t)u * NPOL, acc);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (live && rid >= r0 && rid < r0 + nrr) {
                const float4 q0 = *(const float4 *)(tab8 + px * 8), q1 = *(const float4 *)(tab8 + px * 8 + 4);
                const float tx[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
                const float2 *rr = rbuf + (size_t)(rid - r0) * W * NPOL;
#pragma unroll
                for (int t = 0; t < W; t++) {
                    float2 v[NPOL];
                    load_record<NPOL>(rr + t * NPOL, v);
#pragma unroll
                    for (int p = 0; p < NPOL; p++) {
                        y[p].x = fmaf(tx[t], v[p].x, y[p].x);
                        y[p].y = fmaf(tx[t], v[p].y, y[p].y);
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        if (live) degrid_finish<NPOL>(a, i, y, want_g, gacc);
    }
    if (want_g && a.ant_in_lds) {
        __syncthreads();
        for (int i = tid; i < a.nant; i += nthreads) {
            const float2 v = gacc[i];
            if (v.x != 0.0f) atomicAdd(&a.grad_gains[i].x, v.x);
            if (v.y != 0.0f) atomicAdd(&a.grad_gains[i].y, v.y);
        }
    }
}

} // namespace mwg

