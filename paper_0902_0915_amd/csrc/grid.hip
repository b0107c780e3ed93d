// Gridding kernels: scatter every kept visibility through its W x W kernel footprint onto
// the uv grid (the interpolation onto a regular grid of Section 2.1; "Gridding" in Table 1).
//
// The paper's port replaced scatter loops by gather loops because its GPU had no atomic
// floating-point add (Section 3.2). CDNA4 has fast LDS FP32 atomics, so this gridder keeps
// the scatter but confines it to the chip: visibilities arrive sorted by uv tile (plan
// time), one workgroup owns one tile (or one slice of a heavy tile) staged in LDS with a
// halo of h cells, and only the finished tile goes to HBM, with coalesced stores.
//
// Variant 1 ("tap lanes", W*W <= 64): lane l of a wavefront owns tap (s, t) = (l / W, l % W)
// of the footprint and holds one FP32 accumulator per polarisation component in registers.
// Groups are sorted by cell within the tile, so consecutive groups often share a centre
// cell; the accumulators are only added into the LDS tile when the (wave-uniform) centre
// cell changes. Each group costs one tap read from LDS and 2*npol FMAs per lane.
//
// Variant 3 ("scatter", any W <= 15): one thread per group adds all W*W taps into the LDS
// tile with LDS atomics.
//
// Tile flush: 1 = atomic adds of the tile (with halo) into the zeroed grid in HBM;
//             2 = plain stores of each tile into a per-work-item buffer and a merge pass
//                 that sums the (at most nine) overlapping tiles of every cell.
#include "internal.h"
#include "gridder_core.h"

#include <algorithm>

namespace mwg {

size_t taplanes_lds(int npol, int T, int W, int O, int waves);
size_t collanes_lds(int npol, int T, int W, int O, int waves);
size_t wavetiles_lds(int npol, int T, int W, int O, int waves);
size_t owner_lds(int npol, int T, int W, int O, int waves);
size_t blocktiles_lds(int npol, int T, int W, int O, int waves);
size_t scatter_lds(int npol, int T, int W, int O);
Status ensure_partial(Instance &I, hipStream_t s);

namespace {

constexpr int kFillBlock = 256;

__global__ void k_fill_zero4(float4 *p, int64_t n4) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = i; k < n4; k += stride) p[k] = make_float4(0.f, 0.f, 0.f, 0.f);
}

__global__ void k_fill_zero1(float *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

struct GridArgs {
    const float2 *vis;
    const uint32_t *perm, *spos, *sant, *scode;
    const float *sw;
    const float2 *gains;
    const WorkItem *work;
    const float *taps2d, *tab, *tab8;
    float2 *grid;
    float *partial;  // flush 2
    int nx, ny, T, ntx, W, O, str, plane;
    // The tap table with rows padded to 8 floats, carried in the kernel arguments (constant
    // memory): a wave-uniform row is then a single scalar load.
    float tapk[16 * 8];
    // schedule 2: logical workgroup ranges per XCD (hardware workgroup h runs on XCD h % 8)
    int xcd_start[9];
    int schedule;
    const int2 *coop;  // schedule 3: wave slots
    int accumulate;    // flush 3: add the output tiles to the grid
};

// LDS layout of a tile: 2*NPOL planes (re, im of each polarisation), each R rows of STR
// floats, R = T + W - 1; STR = W (mod 32) makes the 49 lanes of a footprint flush hit 49
// distinct banks. The plane size is padded to a multiple of 4 floats.
__host__ __device__ inline int tile_stride(int R, int W) {
    int s = R;
    while ((s - W) % 32 != 0) s++;
    return s;
}
__host__ __device__ inline int tile_plane(int R, int STR) { return (R * STR + 3) & ~3; }
// Variant 2 puts the 2*npol component planes side by side in one lane set, so the plane
// stride is also congruent to W (mod 32).
__host__ __device__ inline int tile_plane2(int R, int STR, int W) {
    int p = R * STR;
    while ((p - W) % 32 != 0) p++;
    return p;
}

// Multiply a group's visibilities by w * g1 * conj(g2) (when given).
template <int NPOL>
__device__ inline void apply_multiplier(const GridArgs &a, int64_t i, float2 (&v)[NPOL]) {
    if (!a.sw && !a.gains) return;
    float mr = a.sw ? a.sw[i] : 1.0f, mi = 0.0f;
    if (a.gains) {
        const uint32_t an = a.sant[i];
        const float2 g1 = a.gains[an & 0xFFFFu], g2 = a.gains[an >> 16];
        const float gr = g1.x * g2.x + g1.y * g2.y, gi = g1.y * g2.x - g1.x * g2.y;
        mi = mr * gi;
        mr = mr * gr;
    }
#pragma unroll
    for (int p = 0; p < NPOL; p++) {
        const float re = mr * v[p].x - mi * v[p].y, im = mr * v[p].y + mi * v[p].x;
        v[p] = make_float2(re, im);
    }
}

template <int NPOL>
__device__ inline void load_vis(const float2 *vis, uint32_t g, float2 (&v)[NPOL]) {
    const float2 *src = vis + (int64_t)g * NPOL;
    if constexpr (NPOL == 4) {
        const float4 a = ((const float4 *)src)[0], b = ((const float4 *)src)[1];
        v[0] = make_float2(a.x, a.y);
        v[1] = make_float2(a.z, a.w);
        v[2] = make_float2(b.x, b.y);
        v[3] = make_float2(b.z, b.w);
    } else if constexpr (NPOL == 2) {
        const float4 a = ((const float4 *)src)[0];
        v[0] = make_float2(a.x, a.y);
        v[1] = make_float2(a.z, a.w);
    } else {
        v[0] = src[0];
    }
}

// Write the finished LDS tile to HBM (atomic adds, or plain stores into the work item's
// slice of the partial buffer).
template <int NPOL>
__device__ inline void flush_tile(const GridArgs &a, const float *tile, int flush, int tx0, int ty0,
                                  int h, int R, int STR, int PL) {
    const int nthreads = blockDim.x;
    if (flush == 1) {
        for (int idx = threadIdx.x; idx < R * R; idx += nthreads) {
            const int r = idx / R, c = idx - r * R;
            const int gy = ty0 - h + r, gx = tx0 - h + c;
            if (gy < 0 || gy >= a.ny || gx < 0 || gx >= a.nx) continue;
#pragma unroll
            for (int p = 0; p < NPOL; p++) {
                const float re = tile[(2 * p) * PL + r * STR + c];
                const float im = tile[(2 * p + 1) * PL + r * STR + c];
                float *dst = (float *)(a.grid + ((int64_t)p * a.ny + gy) * a.nx + gx);
                if (re != 0.0f) atomicAdd(dst, re);
                if (im != 0.0f) atomicAdd(dst + 1, im);
            }
        }
    } else {
        // cell-major slice: the 2 * NPOL components of a cell contiguous
        float *out = a.partial + (int64_t)blockIdx.x * (2 * NPOL) * R * R;
        for (int idx = threadIdx.x; idx < R * R; idx += nthreads) {
            const int r = idx / R, c = idx - r * R;
            float v[2 * NPOL];
#pragma unroll
            for (int q = 0; q < 2 * NPOL; q++) v[q] = tile[q * PL + r * STR + c];
            store_cell<2 * NPOL>(out + (int64_t)idx * 2 * NPOL, v);
        }
    }
}

// Loads lane's group (index i of the sorted order) and applies its multiplier.
template <int NPOL>
__device__ inline void fetch_group(const GridArgs &a, int64_t i, uint32_t g, float2 (&v)[NPOL]) {
    load_vis<NPOL>(a.vis, g, v);
    apply_multiplier<NPOL>(a, i, v);
}

template <int NPOL>
__global__ __launch_bounds__(1024) void k_grid_taplanes(GridArgs a, int flush) {
    extern __shared__ __align__(16) float smem[];
    const int nthreads = blockDim.x, tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nwaves = nthreads >> 6;
    const WorkItem wk = a.work[blockIdx.x];
    const int T = a.T, W = a.W, h = (W - 1) / 2, R = T + W - 1, STR = a.str, PL = a.plane;
    const int tx0 = (wk.tile % a.ntx) * T, ty0 = (wk.tile / a.ntx) * T;
    const int OO64 = a.O * a.O * 64;
    float *tile = smem;
    float *taps = smem + 2 * NPOL * PL;
    float2 *sv = (float2 *)(taps + OO64) + wave * 64 * NPOL;

    for (int i = tid; i < 2 * NPOL * PL; i += nthreads) tile[i] = 0.0f;
    for (int i = tid; i < OO64; i += nthreads) taps[i] = a.taps2d[i];
    __syncthreads();

    const int n = wk.end - wk.begin;
    const int wb = wk.begin + (int)((int64_t)n * wave / nwaves);
    const int we = wk.begin + (int)((int64_t)n * (wave + 1) / nwaves);
    const int s = lane / W, t = lane - s * W;
    const bool active = lane < W * W;
    const int loff = active ? s * STR + t : 0;
    const float *tapl = taps + lane;
    float acc[2 * NPOL];
#pragma unroll
    for (int k = 0; k < 2 * NPOL; k++) acc[k] = 0.0f;
    int cur = -1;

    // Software pipeline over batches of 64 groups: while batch k is accumulated from LDS,
    // the visibilities of batch k+1 and the permutation entries of batch k+2 are in flight.
    uint32_t gA = (wb + lane < we) ? a.perm[wb + lane] : 0u;
    uint32_t gB = (wb + 64 + lane < we) ? a.perm[wb + 64 + lane] : 0u;
    float2 vn[NPOL];
    if (wb + lane < we) fetch_group<NPOL>(a, wb + lane, gA, vn);

    for (int base = wb; base < we; base += 64) {
        const int cnt = (we - base) < 64 ? (we - base) : 64;
        if (lane < cnt) {
#pragma unroll
            for (int p = 0; p < NPOL; p++) sv[lane * NPOL + p] = vn[p];
        }
        if (base + 64 + lane < we) fetch_group<NPOL>(a, base + 64 + lane, gB, vn);
        gB = (base + 128 + lane < we) ? a.perm[base + 128 + lane] : 0u;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint32_t *spb = a.spos + base;
        for (int j0 = 0; j0 < cnt; j0 += 8) {
            uint32_t pp[8];
#pragma unroll
            for (int u = 0; u < 8; u++) pp[u] = spb[j0 + u]; // uniform; array padded by 64
#pragma unroll
            for (int u = 0; u < 8; u++) {
                if (j0 + u < cnt) {
                    const uint32_t q = pp[u];
                    const int cx = (int)(q & 0xFFFu), cy = (int)((q >> 12) & 0xFFFu);
                    const int ph = (int)((q >> 28) * a.O + ((q >> 24) & 0xFu));
                    const int cell = (cy - ty0) * STR + (cx - tx0);
                    if (cell != cur) {
                        if (cur >= 0 && active) {
#pragma unroll
                            for (int k = 0; k < 2 * NPOL; k++) atomicAdd(&tile[k * PL + cur + loff], acc[k]);
                        }
#pragma unroll
                        for (int k = 0; k < 2 * NPOL; k++) acc[k] = 0.0f;
                        cur = cell;
                    }
                    const float tap = tapl[ph * 64];
                    const float2 *vj = sv + (j0 + u) * NPOL;
#pragma unroll
                    for (int p = 0; p < NPOL; p++) {
                        const float2 v = vj[p];
                        acc[2 * p] = fmaf(tap, v.x, acc[2 * p]);
                        acc[2 * p + 1] = fmaf(tap, v.y, acc[2 * p + 1]);
                    }
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (cur >= 0 && active) {
#pragma unroll
        for (int k = 0; k < 2 * NPOL; k++) atomicAdd(&tile[k * PL + cur + loff], acc[k]);
    }
    __syncthreads();
    flush_tile<NPOL>(a, tile, flush, tx0, ty0, h, R, STR, PL);
}


// Variant 2 ("column lanes", 3 <= W <= 7): lane = (row group sg, component c, column t) with
// c over the 2*NPOL real components of the visibility and NSG = 8/(2*NPOL) row groups, so
// 8*W <= 64 lanes are active (56 for W = 7). A lane forms a = T[px][t] * V_c once per group
// and adds T[py][s] * a into one register accumulator per footprint row s it owns
// (s = sg, sg + NSG, ...). Each group costs the lane two 4-byte LDS reads (V_c and the
// column tap); with NSG = 1 the row taps are wave-uniform scalar loads, otherwise LDS reads.
// As in variant 1 the accumulators go to the LDS tile only when the centre cell changes.
template <int NPOL, int W>
__global__ __launch_bounds__(1024) void k_grid_collanes(GridArgs a, int flush) {
    constexpr int NC = 2 * NPOL;        // real components per group
    constexpr int NSG = 8 / NC;         // row groups
    constexpr int NR = (W + NSG - 1) / NSG; // rows per lane
    extern __shared__ __align__(16) float smem[];
    const int nthreads = blockDim.x, tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nwaves = nthreads >> 6;
    const WorkItem wk = a.work[blockIdx.x];
    const int T = a.T, h = (W - 1) / 2, R = T + W - 1, STR = a.str, PL = a.plane;
    const int tx0 = (wk.tile % a.ntx) * T, ty0 = (wk.tile / a.ntx) * T;
    const int ntab = a.O * 8;           // tap rows padded to 8 floats
    float *tile = smem;
    float *ltab = smem + NC * PL;
    float *sv = ltab + ntab + wave * 64 * NC;

    for (int i = tid; i < NC * PL; i += nthreads) tile[i] = 0.0f;
    for (int i = tid; i < ntab; i += nthreads) ltab[i] = a.tab8[i];
    __syncthreads();

    const int n = wk.end - wk.begin;
    const int wb = wk.begin + (int)((int64_t)n * wave / nwaves);
    const int we = wk.begin + (int)((int64_t)n * (wave + 1) / nwaves);
    const int t = lane % W;
    const int c = (lane / W) % NC;
    const int sg = lane / (W * NC);
    const bool active = lane < W * NC * NSG;
    const int loff = active ? c * PL + sg * STR + t : 0;
    const float *vl = sv + c;          // this lane's component of staged group j: vl[j * NC]
    const float *txl = ltab + t;       // column tap: txl[px * 8]
    float acc[NR];
#pragma unroll
    for (int k = 0; k < NR; k++) acc[k] = 0.0f;
    int cur = -1;

    uint32_t gA = (wb + lane < we) ? a.perm[wb + lane] : 0u;
    uint32_t gB = (wb + 64 + lane < we) ? a.perm[wb + 64 + lane] : 0u;
    float2 vn[NPOL];
    if (wb + lane < we) fetch_group<NPOL>(a, wb + lane, gA, vn);

    for (int base = wb; base < we; base += 64) {
        const int cnt = (we - base) < 64 ? (we - base) : 64;
        if (lane < cnt) {
            float *dst = sv + lane * NC;
#pragma unroll
            for (int p = 0; p < NPOL; p++) {
                dst[2 * p] = vn[p].x;
                dst[2 * p + 1] = vn[p].y;
            }
        }
        if (base + 64 + lane < we) fetch_group<NPOL>(a, base + 64 + lane, gB, vn);
        gB = (base + 128 + lane < we) ? a.perm[base + 128 + lane] : 0u;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint32_t *cb = a.scode + base;
        for (int j0 = 0; j0 < cnt; j0 += 8) {
            uint32_t qq[8];
#pragma unroll
            for (int u = 0; u < 8; u++) qq[u] = cb[j0 + u]; // uniform; array padded by 64
#pragma unroll
            for (int u = 0; u < 8; u++) {
                if (j0 + u < cnt) {
                    const uint32_t q = qq[u];
                    const int cell = (int)(q & 0xFFFFu);
                    const int txo = (int)((q >> 16) & 0xFFu);
                    const int tyo = (int)(q >> 24);
                    if (cell != cur) {
                        if (cur >= 0 && active) {
#pragma unroll
                            for (int k = 0; k < NR; k++)
                                if (sg + NSG * k < W)
                                    atomicAdd(&tile[cur + loff + NSG * k * STR], acc[k]);
                        }
#pragma unroll
                        for (int k = 0; k < NR; k++) acc[k] = 0.0f;
                        cur = cell;
                    }
                    const float va = vl[(j0 + u) * NC] * txl[txo];
                    if constexpr (NSG == 1) {
                        // one 32-byte scalar load of the padded row of row taps
                        const float4 *tyr = (const float4 *)__builtin_assume_aligned(a.tab8 + tyo, 32);
                        const float4 r0 = tyr[0], r1 = tyr[1];
                        const float ty[8] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};
#pragma unroll
                        for (int k = 0; k < NR; k++) acc[k] = fmaf(ty[k], va, acc[k]);
                    } else {
#pragma unroll
                        for (int k = 0; k < NR; k++) {
                            const int sr = sg + NSG * k;
                            const float ty = ltab[tyo + (sr < W ? sr : 0)];
                            acc[k] = fmaf(ty, va, acc[k]);
                        }
                    }
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (cur >= 0 && active) {
#pragma unroll
        for (int k = 0; k < NR; k++)
            if (sg + NSG * k < W) atomicAdd(&tile[cur + loff + NSG * k * STR], acc[k]);
    }
    __syncthreads();
    flush_tile<NPOL>(a, tile, flush, tx0, ty0, h, R, STR, PL);
}


// Variant 4 ("wave tiles", 3 <= W <= 7): the lane layout of variant 2, but every wavefront
// owns one work item and a private haloed tile in LDS (small tiles, T = 8 or 16). With no
// other wavefront touching its tile, the accumulator flush on a cell change is a plain
// LDS read-add-write instead of an LDS float atomic (which costs ~40x more on this chip).
// The finished tile goes to HBM by atomic adds (flush 1) or into the work item's slice of
// the partial buffer, summed by the merge pass (flush 2).
template <int NPOL, int W>
__global__ __launch_bounds__(1024) void k_grid_wavetiles(GridArgs a, int flush, int nwork) {
    constexpr int NC = 2 * NPOL;
    extern __shared__ __align__(16) float smem[];
    const int nthreads = blockDim.x, tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nwaves = nthreads >> 6;
    const int ntab = a.O * 8;
    float *ltab = smem;
    for (int i = tid; i < ntab; i += nthreads) ltab[i] = a.tab8[i];
    __syncthreads();
    int lb = blockIdx.x;
    if (a.schedule == 2) {
        const int x = blockIdx.x & 7;
        lb = a.xcd_start[x] + (blockIdx.x >> 3);
        if (lb >= a.xcd_start[x + 1]) return;
    }
    const int widx = lb * nwaves + wave;
    if (widx >= nwork) return;
    const int R = a.T + W - 1;
    const int per_wave = wavetile_per_wave(NC, a.plane);
    ItemCtx c;
    c.sv = smem + ntab + wave * per_wave;
    c.tile = c.sv + kStageFloats;
    for (int i = lane; i < NC * a.plane; i += 64) c.tile[i] = 0.0f;
    const WorkItem wk = a.work[widx];
    c.vis = a.vis;
    c.gains = a.gains;
    c.perm = a.perm;
    c.scode = a.scode;
    c.sant = a.sant;
    c.sw = a.sw;
    c.tapk = a.tapk;
    c.ltab = ltab;
    c.grid = a.grid;
    c.partial = flush == 2 ? a.partial + (int64_t)widx * NC * R * R : nullptr;
    c.accumulate = a.accumulate;
    c.wb = wk.begin;
    c.we = wk.end;
    c.tx0 = (wk.tile % a.ntx) * a.T;
    c.ty0 = (wk.tile / a.ntx) * a.T;
    c.T = a.T;
    c.STR = a.str;
    c.PL = a.plane;
    c.nx = a.nx;
    c.ny = a.ny;
    c.flush = flush;
    wavetile_item<NPOL, W>(c, lane);
}

// Variant 6: the wave-tile gridder over the plan's block-padded work list (schedule 1).
template <int NPOL, int W>
__global__ __launch_bounds__(1024) void k_grid_blocktiles(GridArgs a, int flush, int nwork) {
    constexpr int NC = 2 * NPOL;
    extern __shared__ __align__(16) float smem[];
    const int nthreads = blockDim.x, tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nwaves = nthreads >> 6;
    const int ntab = a.O * 8;
    float *ltab = smem;
    for (int i = tid; i < ntab; i += nthreads) ltab[i] = a.tab8[i];
    __syncthreads();
    const int widx = blockIdx.x * nwaves + wave;
    if (widx >= nwork) return;
    const int R = a.T + W - 1;
    ItemCtx c;
    c.sv = smem + ntab + wave * blocktile_per_wave(NC, a.plane);
    c.tile = c.sv + blocktile_stage_floats(NC);
    for (int i = lane; i < NC * a.plane; i += 64) c.tile[i] = 0.0f;
    const WorkItem wk = a.work[widx];
    c.vis = a.vis;
    c.gains = a.gains;
    c.perm = a.perm;
    c.scode = a.scode;
    c.sant = a.sant;
    c.sw = a.sw;
    c.tapk = a.tapk;
    c.ltab = ltab;
    c.grid = a.grid;
    c.partial = flush == 2 ? a.partial + (int64_t)widx * NC * R * R : nullptr;
    c.accumulate = a.accumulate;
    c.wb = wk.begin;
    c.we = wk.end;
    c.tx0 = (wk.tile % a.ntx) * a.T;
    c.ty0 = (wk.tile / a.ntx) * a.T;
    c.T = a.T;
    c.STR = a.str;
    c.PL = a.plane;
    c.nx = a.nx;
    c.ny = a.ny;
    c.flush = flush;
    blocktile_item<NPOL, W>(c, lane);
}

// Schedule 3 of variant 4: the waves of a workgroup share its items. Slot j of the
// workgroup (wave j) grids part k of the nsub equal parts of item coop[j].x into its private
// tile; after a barrier the workgroup sums each item's nsub tiles in wave order into the
// item's partial slice. The waves of one item work on neighbouring cell rows of the same tile
// at the same time, so a visibility line that feeds cells in several rows is fetched once
// into the cache for all of them rather than once per cell row.
template <int NPOL, int W>
__global__ __launch_bounds__(1024) void k_grid_wavetiles_coop(GridArgs a) {
    constexpr int NC = 2 * NPOL;
    extern __shared__ __align__(16) float smem[];
    const int nthreads = blockDim.x, tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nwaves = nthreads >> 6;
    const int ntab = a.O * 8;
    float *ltab = smem;
    for (int i = tid; i < ntab; i += nthreads) ltab[i] = a.tab8[i];
    const int R = a.T + W - 1;
    const int per_wave = wavetile_per_wave(NC, a.plane);
    float *mytile = smem + ntab + wave * per_wave + kStageFloats;
    for (int i = lane; i < NC * a.plane; i += 64) mytile[i] = 0.0f;
    __syncthreads();
    const int2 *slots = a.coop + (int64_t)blockIdx.x * nwaves;
    const int2 task = slots[wave];
    const int item = __builtin_amdgcn_readfirstlane(task.x);
    if (item >= 0) {
        const int k = __builtin_amdgcn_readfirstlane(task.y & 0xFF);
        const int nsub = __builtin_amdgcn_readfirstlane(task.y >> 8);
        const WorkItem wk = a.work[item];
        const int64_t n = (int64_t)wk.end - wk.begin;
        ItemCtx c;
        c.sv = smem + ntab + wave * per_wave;
        c.tile = mytile;
        c.vis = a.vis;
        c.gains = a.gains;
        c.perm = a.perm;
        c.scode = a.scode;
        c.sant = a.sant;
        c.sw = a.sw;
        c.tapk = a.tapk;
        c.ltab = ltab;
        c.grid = a.grid;
        c.partial = nullptr;
        c.wb = __builtin_amdgcn_readfirstlane((int)(wk.begin + n * k / nsub));
        c.we = __builtin_amdgcn_readfirstlane((int)(wk.begin + n * (k + 1) / nsub));
        c.tx0 = (wk.tile % a.ntx) * a.T;
        c.ty0 = (wk.tile / a.ntx) * a.T;
        c.T = a.T;
        c.STR = a.str;
        c.PL = a.plane;
        c.nx = a.nx;
        c.ny = a.ny;
        c.flush = 0;
        wavetile_item<NPOL, W>(c, lane);
    }
    __syncthreads();
    // every item of the workgroup: its first wave's slot says how many tiles to sum
    const int RR = R * R;
    for (int j = 0; j < nwaves; j++) {
        const int2 tj = slots[j];
        const int it = __builtin_amdgcn_readfirstlane(tj.x);
        if (it < 0 || (tj.y & 0xFF) != 0) continue;
        const int nsub = __builtin_amdgcn_readfirstlane(tj.y >> 8);
        const float *t0 = smem + ntab + j * per_wave + kStageFloats;
        float *out = a.partial + (int64_t)it * NC * RR;
        for (int idx = tid; idx < NC * RR; idx += nthreads) {  // cell-major, as the merge reads it
            const int rr = idx / NC, q = idx - rr * NC;
            const int r = rr / R, col = rr - r * R;
            const int off = q * a.plane + r * a.str + col;
            float v = t0[off];
            for (int m = 1; m < nsub; m++) v += t0[m * per_wave + off];
            out[idx] = v;
        }
    }
}

template <int NPOL>
__global__ __launch_bounds__(1024) void k_grid_scatter(GridArgs a, int flush) {
    extern __shared__ __align__(16) float smem[];
    const int nthreads = blockDim.x, tid = threadIdx.x;
    const WorkItem wk = a.work[blockIdx.x];
    const int T = a.T, W = a.W, h = (W - 1) / 2, R = T + W - 1, STR = a.str, PL = a.plane;
    const int tx0 = (wk.tile % a.ntx) * T, ty0 = (wk.tile / a.ntx) * T;
    float *tile = smem;
    float *tab = smem + 2 * NPOL * PL;
    for (int i = tid; i < 2 * NPOL * PL; i += nthreads) tile[i] = 0.0f;
    for (int i = tid; i < a.O * W; i += nthreads) tab[i] = a.tab[i];
    __syncthreads();
    for (int64_t i = wk.begin + tid; i < wk.end; i += nthreads) {
        float2 v[NPOL];
        load_vis<NPOL>(a.vis, a.perm[i], v);
        apply_multiplier<NPOL>(a, i, v);
        const uint32_t pp = a.spos[i];
        const int cx = (int)(pp & 0xFFFu), cy = (int)((pp >> 12) & 0xFFFu);
        const int px = (int)((pp >> 24) & 0xFu), py = (int)(pp >> 28);
        const int o = (cy - ty0) * STR + (cx - tx0);
        for (int sy = 0; sy < W; sy++) {
            const float ty = tab[py * W + sy];
            for (int sx = 0; sx < W; sx++) {
                const float tap = ty * tab[px * W + sx];
                const int c = o + sy * STR + sx;
#pragma unroll
                for (int p = 0; p < NPOL; p++) {
                    atomicAdd(&tile[(2 * p) * PL + c], tap * v[p].x);
                    atomicAdd(&tile[(2 * p + 1) * PL + c], tap * v[p].y);
                }
            }
        }
    }
    __syncthreads();
    flush_tile<NPOL>(a, tile, flush, tx0, ty0, h, R, STR, PL);
}

// Merge pass of flush 2: every grid cell sums the partial tiles of all work items whose
// (haloed) tile covers it, in a fixed order.
// One launch covers the listed blocks that some work item reaches (merged), then the nzero
// listed blocks that none reaches (zeroed), one block per workgroup. The first 8 * chunk
// workgroups merge, chunk = ceil(nblocks / 8): they are dealt to the 8 XCDs in turn and
// workgroup w takes list entry (w mod 8) * chunk + w / 8, so each XCD merges one contiguous
// band of the list and the blocks that read the same partial tiles share that XCD's L2.
template <int NPOL>
__global__ __launch_bounds__(kMergeB * kMergeB) void k_merge(float2 *grid, const float *partial,
                                                              const int32_t *tile_work, const int32_t *work_ids,
                                                              const int32_t *blocks, int nblocks, int nzero, int nx,
                                                              int ny, int lgT, int ntx, int nty, int W, int accumulate) {
    __shared__ int2 rng[kMergeTiles];
    __shared__ int fid[kMergeTiles];
    const int bpr = (nx + kMergeB - 1) / kMergeB, h = (W - 1) / 2;
    const int tid = threadIdx.x;
    const int chunk = (nblocks + 7) / 8;
    if ((int)blockIdx.x >= 8 * chunk) {
        const int z = (int)blockIdx.x - 8 * chunk;
        if (z >= nzero) return;
        const int b = blocks[nblocks + z], by = b / bpr, bx = b - by * bpr;
        zero_block<NPOL>(grid, nx, ny, bx * kMergeB, by * kMergeB);
        return;
    }
    const int e = (int)(blockIdx.x & 7u) * chunk + (int)(blockIdx.x >> 3);
    if (e >= nblocks) return;
    const int b = blocks[e], by = b / bpr, bx = b - by * bpr;
    const int x0 = bx * kMergeB, y0 = by * kMergeB;
    const MergeBounds m = merge_bounds(x0, y0, h, lgT, ntx, nty);
    if (tid < 32) merge_stage(tile_work, work_ids, ntx, m, tid, rng, fid);
    __syncthreads();
    merge_cell<NPOL>(grid, partial, work_ids, nx, ny, lgT, W, accumulate, m, rng, fid, x0 + (tid & (kMergeB - 1)),
                     y0 + tid / kMergeB);
}

template <int NPOL>
Status launch_grid_npol(Instance &I, GridArgs &a, int accumulate, hipStream_t s, float *partial_in = nullptr,
                        size_t partial_cap = 0) {
    const Launch &L = I.L;
    const int R = L.tile + I.W - 1;
    a.str = (L.variant == 4 || L.variant == 6) ? R : tile_stride(R, I.W);
    a.plane = (L.variant == 2 || L.variant == 4 || L.variant == 6) ? tile_plane2(R, a.str, I.W)
                                                                    : tile_plane(R, a.str);
    const int flush = L.flush;
    if (partial_in) {
        const size_t need = sizeof(float) * (size_t)std::max(I.nwork, 1) * 2 * I.npol * R * R;
        if (flush == 2 && need > partial_cap)
            return make_error(MW_ERR_UNSUPPORTED,
                              "the merge flush of this plan needs %zu B of scratch, more than the %zu B available",
                              need, partial_cap);
        a.partial = partial_in;
    } else {
        if (flush == 2) MWG_TRY(ensure_partial(I, s));
        a.partial = I.partial;
    }
    int nwork = I.nwork;
    if (flush == 3) {
        // owner tiles: the work list, codes and sorted arrays of the (output tile, group) pairs
        if (L.variant != 4 || I.owner_tile != L.tile)
            return make_error(MW_ERR_STATE, "flush 3 needs the owner-tile schedule of the wave-tile gridder");
        a.work = I.owork;
        a.perm = I.pperm;
        a.scode = I.pcode;
        a.sw = I.psw;
        a.sant = I.psant;
        a.str = owner_span(L.tile, I.W);
        a.plane = owner_plane(L.tile, I.W);
        a.accumulate = accumulate;
        nwork = I.nowork;
    }
    if (flush == 1 && !accumulate)
        MWG_TRY(launch_fill_zero(a.grid, sizeof(float2) * (size_t)NPOL * I.nx * I.ny, s));
    if (I.timing) MWG_HIP(hipEventRecord(I.tev[0], s));
    if (nwork > 0) {
        if (L.variant == 1) {
            const size_t lds = taplanes_lds(NPOL, L.tile, I.W, I.O, L.wg_waves);
            if (lds > 160 * 1024) return make_error(MW_ERR_UNSUPPORTED, "tile needs %zu B of LDS", lds);
            hipLaunchKernelGGL(k_grid_taplanes<NPOL>, dim3(I.nwork), dim3(64 * L.wg_waves), lds, s, a, flush);
        } else if (L.variant == 2) {
            const size_t lds = collanes_lds(NPOL, L.tile, I.W, I.O, L.wg_waves);
            if (lds > 160 * 1024) return make_error(MW_ERR_UNSUPPORTED, "tile needs %zu B of LDS", lds);
            const dim3 g(I.nwork), b(64 * L.wg_waves);
            switch (I.W) {
            case 3: hipLaunchKernelGGL((k_grid_collanes<NPOL, 3>), g, b, lds, s, a, flush); break;
            case 5: hipLaunchKernelGGL((k_grid_collanes<NPOL, 5>), g, b, lds, s, a, flush); break;
            case 7: hipLaunchKernelGGL((k_grid_collanes<NPOL, 7>), g, b, lds, s, a, flush); break;
            default: return make_error(MW_ERR_UNSUPPORTED, "variant 2 needs W in {3, 5, 7}");
            }
        } else if (L.variant == 4) {
            const size_t lds = flush == 3 ? owner_lds(NPOL, L.tile, I.W, I.O, L.wg_waves)
                                          : wavetiles_lds(NPOL, L.tile, I.W, I.O, L.wg_waves);
            if (lds > 160 * 1024) return make_error(MW_ERR_UNSUPPORTED, "tile needs %zu B of LDS", lds);
            if (L.schedule == 3) {
                a.coop = I.coop;
                const dim3 g(I.coop_wgs), b(64 * L.wg_waves);
                switch (I.W) {
                case 3: hipLaunchKernelGGL((k_grid_wavetiles_coop<NPOL, 3>), g, b, lds, s, a); break;
                case 5: hipLaunchKernelGGL((k_grid_wavetiles_coop<NPOL, 5>), g, b, lds, s, a); break;
                case 7: hipLaunchKernelGGL((k_grid_wavetiles_coop<NPOL, 7>), g, b, lds, s, a); break;
                default: return make_error(MW_ERR_UNSUPPORTED, "variant 4 needs W in {3, 5, 7}");
                }
            } else {
                const dim3 g(L.schedule == 2 ? 8 * I.xcd_wgs : (nwork + L.wg_waves - 1) / L.wg_waves),
                    b(64 * L.wg_waves);
                a.schedule = L.schedule;
                for (int x = 0; x < 9; x++) a.xcd_start[x] = I.xcd_start[x];
                switch (I.W) {
                case 3: hipLaunchKernelGGL((k_grid_wavetiles<NPOL, 3>), g, b, lds, s, a, flush, nwork); break;
                case 5: hipLaunchKernelGGL((k_grid_wavetiles<NPOL, 5>), g, b, lds, s, a, flush, nwork); break;
                case 7: hipLaunchKernelGGL((k_grid_wavetiles<NPOL, 7>), g, b, lds, s, a, flush, nwork); break;
                default: return make_error(MW_ERR_UNSUPPORTED, "variant 4 needs W in {3, 5, 7}");
                }
            }
        } else if (L.variant == 6) {
            // the block-padded list replaces the sorted arrays (same items, same partial slices)
            if (!I.bwork || I.block_tile != L.tile)
                return make_error(MW_ERR_STATE, "variant 6 needs the plan's block-padded schedule");
            a.work = I.bwork;
            a.perm = I.bperm;
            a.scode = I.bcode;
            a.sw = I.bsw;
            a.sant = I.bsant;
            const size_t lds = blocktiles_lds(NPOL, L.tile, I.W, I.O, L.wg_waves);
            if (lds > 160 * 1024) return make_error(MW_ERR_UNSUPPORTED, "tile needs %zu B of LDS", lds);
            const dim3 g((nwork + L.wg_waves - 1) / L.wg_waves), b(64 * L.wg_waves);
            switch (I.W) {
            case 3: hipLaunchKernelGGL((k_grid_blocktiles<NPOL, 3>), g, b, lds, s, a, flush, nwork); break;
            case 5: hipLaunchKernelGGL((k_grid_blocktiles<NPOL, 5>), g, b, lds, s, a, flush, nwork); break;
            case 7: hipLaunchKernelGGL((k_grid_blocktiles<NPOL, 7>), g, b, lds, s, a, flush, nwork); break;
            default: return make_error(MW_ERR_UNSUPPORTED, "variant 6 needs W in {3, 5, 7}");
            }
        } else {
            const size_t lds = scatter_lds(NPOL, L.tile, I.W, I.O);
            if (lds > 160 * 1024) return make_error(MW_ERR_UNSUPPORTED, "tile needs %zu B of LDS", lds);
            hipLaunchKernelGGL(k_grid_scatter<NPOL>, dim3(I.nwork), dim3(64 * L.wg_waves), lds, s, a, flush);
        }
        MWG_HIP(hipGetLastError());
    }
    if (I.timing) MWG_HIP(hipEventRecord(I.tev[1], s));
    if (flush == 3 && !accumulate) MWG_TRY(launch_zero_tiles(I, a.grid, s));
    if (flush == 2) {
        const int nzero = accumulate ? 0 : I.n_zblocks;
        if (I.n_mblocks + nzero > 0) {
            const int chunk = (I.n_mblocks + 7) / 8;
            hipLaunchKernelGGL(k_merge<NPOL>, dim3(8 * chunk + nzero), dim3(kMergeB * kMergeB), 0, s, a.grid,
                               (const float *)a.partial, (const int32_t *)I.tile_work, (const int32_t *)I.work_ids,
                               (const int32_t *)I.mblocks, I.n_mblocks, nzero, I.nx, I.ny, ilog2(L.tile), I.ntx,
                               I.nty, I.W, accumulate);
            MWG_HIP(hipGetLastError());
        }
    }
    if (I.timing) {
        MWG_HIP(hipEventRecord(I.tev[2], s));
        I.timed = true;
    }
    return Status::Ok();
}

} // namespace

size_t taplanes_lds(int npol, int T, int W, int O, int waves) {
    const int R = T + W - 1, STR = tile_stride(R, W), PL = tile_plane(R, STR);
    return 4 * ((size_t)2 * npol * PL + (size_t)O * O * 64) + (size_t)waves * 64 * (8 * npol);
}

size_t collanes_lds(int npol, int T, int W, int O, int waves) {
    const int R = T + W - 1, STR = tile_stride(R, W), PL = tile_plane2(R, STR, W);
    return 4 * ((size_t)2 * npol * PL + (size_t)O * 8) + (size_t)waves * 64 * 8 * npol;
}

size_t wavetiles_lds(int npol, int T, int W, int O, int waves) {
    const int R = T + W - 1, PL = tile_plane2(R, R, W);
    return 4 * ((size_t)O * 8 + (size_t)waves * wavetile_per_wave(2 * npol, PL));
}

size_t blocktiles_lds(int npol, int T, int W, int O, int waves) {
    const int R = T + W - 1, PL = tile_plane2(R, R, W);
    return 4 * ((size_t)O * 8 + (size_t)waves * blocktile_per_wave(2 * npol, PL));
}

size_t owner_lds(int npol, int T, int W, int O, int waves) {
    return 4 * ((size_t)O * 8 + (size_t)waves * wavetile_per_wave(2 * npol, owner_plane(T, W)));
}

size_t scatter_lds(int npol, int T, int W, int O) {
    const int R = T + W - 1, STR = tile_stride(R, W), PL = tile_plane(R, STR);
    return 4 * ((size_t)2 * npol * PL + (size_t)O * W);
}

// The merge flush's per-work-item tile buffer, sized for the current schedule.
Status ensure_partial(Instance &I, hipStream_t s) {
    (void)s;
    const int R = I.L.tile + I.W - 1;
    const size_t need = sizeof(float) * (size_t)std::max(I.nwork, 1) * 2 * I.npol * R * R;
    if (I.partial_bytes < need) {
        void *p;
        MWG_TRY(I.arena.alloc(&p, need));
        I.partial = (float *)p;
        I.partial_bytes = need;
    }
    return Status::Ok();
}

Status launch_fill_zero(void *ptr, size_t nbytes, hipStream_t s) {
    if (nbytes == 0) return Status::Ok();
    if (((uintptr_t)ptr % 16) == 0 && nbytes % 16 == 0) {
        const int64_t n4 = (int64_t)(nbytes / 16);
        const int64_t blocks = std::min<int64_t>((n4 + kFillBlock - 1) / kFillBlock, 1 << 16);
        hipLaunchKernelGGL(k_fill_zero4, dim3((unsigned)blocks), dim3(kFillBlock), 0, s, (float4 *)ptr, n4);
    } else {
        const int64_t n = (int64_t)(nbytes / 4);
        hipLaunchKernelGGL(k_fill_zero1, dim3((unsigned)((n + kFillBlock - 1) / kFillBlock)),
                           dim3(kFillBlock), 0, s, (float *)ptr, n);
    }
    MWG_HIP(hipGetLastError());
    return Status::Ok();
}

Status launch_grid(Instance &I, const float2 *vis, const float2 *gains, float2 *grid, int accumulate,
                   hipStream_t s) {
    return launch_grid_into(I, vis, gains, grid, accumulate, nullptr, 0, s);
}

Status launch_grid_into(Instance &I, const float2 *vis, const float2 *gains, float2 *grid, int accumulate,
                        float *partial, size_t partial_cap, hipStream_t s) {
    if (I.stacks) return launch_grid_stack(I, vis, gains, grid, accumulate, s);
    GridArgs a{};
    a.vis = vis;
    a.perm = I.perm;
    a.spos = I.spos;
    a.scode = I.scode;
    a.sant = I.sant;
    a.sw = I.sw;
    a.gains = gains;
    a.work = I.work;
    a.taps2d = I.taps2d;
    a.tab = I.tab;
    a.tab8 = I.tab8;
    a.grid = grid;
    for (int i = 0; i < 16 * 8; i++) a.tapk[i] = 0.0f;
    if (!I.stacks && I.W <= 8)
        for (int r = 0; r < I.O; r++)
            for (int t = 0; t < I.W; t++) a.tapk[r * 8 + t] = I.h_tab[(size_t)r * I.W + t];
    a.nx = I.nx;
    a.ny = I.ny;
    a.T = I.L.tile;
    a.ntx = I.ntx;
    a.W = I.W;
    a.O = I.O;
    switch (I.npol) {
    case 1: return launch_grid_npol<1>(I, a, accumulate, s, partial, partial_cap);
    case 2: return launch_grid_npol<2>(I, a, accumulate, s, partial, partial_cap);
    case 4: return launch_grid_npol<4>(I, a, accumulate, s, partial, partial_cap);
    default: return make_error(MW_ERR_UNSUPPORTED, "npol %d", I.npol);
    }
}

} // namespace mwg
