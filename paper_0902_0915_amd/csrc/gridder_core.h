// Shared device code of the wave-tile gridder (variant 4), used by the single-instance
// kernel (grid.hip) and the batched persistent kernel (batched.hip).
#pragma once

#include "internal.h"

namespace mwg {

// Everything one wavefront needs to grid one work item into its private LDS tile.
struct ItemCtx {
    const float2 *vis, *gains;
    const uint32_t *perm, *scode, *sant;
    const float *sw;
    const float *tapk;   // tap rows padded to 8 floats, in constant (kernel-argument) memory
    const float *ltab;   // the same table in LDS
    float *tile, *sv;    // this wave's LDS tile (NC planes of PL floats) and staging area
    float2 *grid;        // flush 1 target
    float *partial;      // flush 2 target: this work item's slice
    int wb, we, tx0, ty0, T, STR, PL, nx, ny, flush;
};

template <int NPOL>
__device__ inline void core_fetch(const ItemCtx &c, int i, uint32_t g, float2 (&v)[NPOL]) {
    const float2 *src = c.vis + (int64_t)g * NPOL;
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
    if (!c.sw && !c.gains) return;
    float mr = c.sw ? c.sw[i] : 1.0f, mi = 0.0f;
    if (c.gains) {
        const uint32_t an = c.sant[i];
        const float2 g1 = c.gains[an & 0xFFFFu], g2 = c.gains[an >> 16];
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

// Adds a lane's row accumulators into its wave-private LDS tile: all reads are issued
// before any write (the rows are distinct addresses), so the flush costs one LDS round trip.
template <int NR, int NSG, int W>
__device__ inline void wave_tile_add(float *p, int STR, int sg, const float (&acc)[NR]) {
    float old[NR];
#pragma unroll
    for (int k = 0; k < NR; k++) old[k] = (sg + NSG * k < W) ? p[NSG * k * STR] : 0.0f;
#pragma unroll
    for (int k = 0; k < NR; k++)
        if (sg + NSG * k < W) p[NSG * k * STR] = old[k] + acc[k];
}

// Grids work item c with this wavefront (lanes as in variant 2) into its private tile and
// writes the tile out. The tile must be zero on entry.
template <int NPOL, int W>
__device__ inline void wavetile_item(const ItemCtx &c, int lane) {
    constexpr int NC = 2 * NPOL;
    constexpr int NSG = 8 / NC;
    constexpr int NR = (W + NSG - 1) / NSG;
    const int T = c.T, h = (W - 1) / 2, R = T + W - 1, STR = c.STR, PL = c.PL;
    const int tx0 = c.tx0, ty0 = c.ty0;
    float *tile = c.tile, *sv = c.sv;
    const float *ltab = c.ltab;
    const int wb = c.wb, we = c.we;
    const int t = lane % W;
    const int cc = (lane / W) % NC;
    const int sg = lane / (W * NC);
    const bool active = lane < W * NC * NSG;
    const int loff = active ? cc * PL + sg * STR + t : 0;
    const float *vl = sv + cc;
    const float *txl = ltab + t;
    float acc[NR];
#pragma unroll
    for (int k = 0; k < NR; k++) acc[k] = 0.0f;
    int cur = -1;

    // Software pipeline over batches of 64 groups. Lane j holds group j's code in a VGPR
    // (read into a scalar register per group with v_readlane) and stages its visibilities
    // in LDS; the next batch's codes and visibilities and the permutation two batches ahead
    // are in flight while a batch is accumulated.
    uint32_t gA = (wb + lane < we) ? c.perm[wb + lane] : 0u;
    uint32_t gB = (wb + 64 + lane < we) ? c.perm[wb + 64 + lane] : 0u;
    uint32_t qn = (wb + lane < we) ? c.scode[wb + lane] : 0u;
    float2 vn[NPOL];
    if (wb + lane < we) core_fetch<NPOL>(c, wb + lane, gA, vn);

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
        const uint32_t qcur = qn;
        if (base + 64 + lane < we) {
            core_fetch<NPOL>(c, base + 64 + lane, gB, vn);
            qn = c.scode[base + 64 + lane];
        }
        gB = (base + 128 + lane < we) ? c.perm[base + 128 + lane] : 0u;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // Runs of equal centre cell: lane j flags whether group j starts a new run.
        const int cellj = (int)(qcur & 0xFFFFu);
        int prevj = __shfl_up(cellj, 1, 64);
        if (lane == 0) prevj = cur;
        const uint64_t starts = __ballot(lane < cnt && cellj != prevj);
        int j = 0;
        while (j < cnt) {
            const uint64_t later = (j + 1 < 64) ? (starts >> (j + 1)) : 0ull;
            const int e = later ? (j + 1 + (int)__builtin_ctzll(later)) : cnt;
            if ((starts >> j) & 1ull) {
                if (cur >= 0 && active) wave_tile_add<NR, NSG, W>(tile + cur + loff, STR, sg, acc);
#pragma unroll
                for (int k = 0; k < NR; k++) acc[k] = 0.0f;
                cur = (int)((uint32_t)__builtin_amdgcn_readlane((int)qcur, j) & 0xFFFFu);
            }
            // branch-free accumulation over the run [j, e), four groups per step so that
            // their LDS and scalar loads share one wait
            int jj = j;
            for (; jj + 4 <= e; jj += 4) {
                uint32_t q[4];
                float va[4];
#pragma unroll
                for (int u = 0; u < 4; u++) q[u] = (uint32_t)__builtin_amdgcn_readlane((int)qcur, jj + u);
#pragma unroll
                for (int u = 0; u < 4; u++) va[u] = vl[(jj + u) * NC] * txl[(q[u] >> 16) & 0xFFu];
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const int tyo = (int)(q[u] >> 24);
                    if constexpr (NSG == 1) {
                        const float *tyr = c.tapk + tyo;
#pragma unroll
                        for (int k = 0; k < NR; k++) acc[k] = fmaf(tyr[k], va[u], acc[k]);
                    } else {
#pragma unroll
                        for (int k = 0; k < NR; k++) {
                            const int sr = sg + NSG * k;
                            acc[k] = fmaf(ltab[tyo + (sr < W ? sr : 0)], va[u], acc[k]);
                        }
                    }
                }
            }
            for (; jj < e; jj++) {
                const uint32_t q = (uint32_t)__builtin_amdgcn_readlane((int)qcur, jj);
                const int tyo = (int)(q >> 24);
                const float va = vl[jj * NC] * txl[(q >> 16) & 0xFFu];
                if constexpr (NSG == 1) {
                    const float *tyr = c.tapk + tyo;
#pragma unroll
                    for (int k = 0; k < NR; k++) acc[k] = fmaf(tyr[k], va, acc[k]);
                } else {
#pragma unroll
                    for (int k = 0; k < NR; k++) {
                        const int sr = sg + NSG * k;
                        acc[k] = fmaf(ltab[tyo + (sr < W ? sr : 0)], va, acc[k]);
                    }
                }
            }
            j = e;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (cur >= 0 && active) wave_tile_add<NR, NSG, W>(tile + cur + loff, STR, sg, acc);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // this wave's tile to HBM
    if (c.flush == 1) {
        for (int idx = lane; idx < R * R; idx += 64) {
            const int r = idx / R, col = idx - r * R;
            const int gy = ty0 - h + r, gx = tx0 - h + col;
            if (gy < 0 || gy >= c.ny || gx < 0 || gx >= c.nx) continue;
#pragma unroll
            for (int p = 0; p < NPOL; p++) {
                const float re = tile[(2 * p) * PL + r * STR + col];
                const float im = tile[(2 * p + 1) * PL + r * STR + col];
                float *dst = (float *)(c.grid + ((int64_t)p * c.ny + gy) * c.nx + gx);
                if (re != 0.0f) atomicAdd(dst, re);
                if (im != 0.0f) atomicAdd(dst + 1, im);
            }
        }
    } else {
        float *out = c.partial;
        for (int idx = lane; idx < R * R; idx += 64) {
            const int r = idx / R, col = idx - r * R;
#pragma unroll
            for (int q = 0; q < NC; q++) out[(int64_t)q * R * R + idx] = tile[q * PL + r * STR + col];
        }
    }
}

// The merge pass over one block of kMergeB x kMergeB cells, run by kMergeB^2 threads (one
// cell each). Every cell is the sum over the partial tiles of the work items whose haloed
// tile covers it, in a fixed order (tile row, tile column, then the tile's work items), so
// the result is bit-reproducible. The work-item ranges of the tiles that can cover the
// block are staged in LDS first: a span of 16 + 2h cells meets at most
// floor((15 + 2h) / T) + 2 tiles per axis, which is 5 for T >= 8 and h <= 7 (W <= 15). A
// block that no work item reaches is written as zeros (or left alone when accumulating).
constexpr int kMergeB = 16;
constexpr int kMergeTiles = 25;

template <int NPOL>
__device__ inline void merge_block(float2 *grid, const float *partial, const int32_t *tile_work,
                                   const int32_t *work_ids, int nx, int ny, int lgT, int ntx, int nty,
                                   int W, int accumulate, int x0, int y0, int2 *rng) {
    constexpr int NC = 2 * NPOL;
    const int T = 1 << lgT, h = (W - 1) / 2, R = T + W - 1;
    const int tid = threadIdx.x;
    const int tx_lo = max(0, x0 - h) >> lgT, tx_hi = min(ntx - 1, (x0 + kMergeB - 1 + h) >> lgT);
    const int ty_lo = max(0, y0 - h) >> lgT, ty_hi = min(nty - 1, (y0 + kMergeB - 1 + h) >> lgT);
    const int ntxb = tx_hi - tx_lo + 1, ntyb = ty_hi - ty_lo + 1;
    if (tid < ntxb * ntyb) {
        const int t = (ty_lo + tid / ntxb) * ntx + tx_lo + tid % ntxb;
        rng[tid] = make_int2(tile_work[t], tile_work[t + 1]);
    }
    __syncthreads();
    int total = 0;
    for (int i = 0; i < ntxb * ntyb; i++) total += rng[i].y - rng[i].x;
    const int x = x0 + (tid & (kMergeB - 1)), y = y0 + tid / kMergeB;
    if (x >= nx || y >= ny) return;
    if (total == 0 && accumulate) return;
    float acc[NC];
#pragma unroll
    for (int q = 0; q < NC; q++) acc[q] = 0.0f;
    if (total > 0) {
        const int txc = x >> lgT, tyc = y >> lgT;
        for (int dy = -1; dy <= 1; dy++) {
            const int tty = tyc + dy;
            if (tty < ty_lo || tty > ty_hi) continue;
            const int r = y - (tty * T - h);
            if (r < 0 || r >= R) continue;
            for (int dx = -1; dx <= 1; dx++) {
                const int ttx = txc + dx;
                if (ttx < tx_lo || ttx > tx_hi) continue;
                const int c = x - (ttx * T - h);
                if (c < 0 || c >= R) continue;
                const int2 rg = rng[(tty - ty_lo) * ntxb + (ttx - tx_lo)];
                for (int k = rg.x; k < rg.y; k++) {
                    const float *src = partial + (int64_t)work_ids[k] * NC * R * R + r * R + c;
#pragma unroll
                    for (int q = 0; q < NC; q++) acc[q] += src[(int64_t)q * R * R];
                }
            }
        }
    }
#pragma unroll
    for (int p = 0; p < NPOL; p++) {
        float2 *dst = grid + ((int64_t)p * ny + y) * nx + x;
        float2 v = make_float2(acc[2 * p], acc[2 * p + 1]);
        if (accumulate) {
            const float2 o = *dst;
            v.x += o.x;
            v.y += o.y;
        }
        *dst = v;
    }
}

} // namespace mwg
