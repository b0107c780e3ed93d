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
    float2 *grid;        // flush 1 and 3 target
    float *partial;      // flush 2 target: this work item's slice
    int wb, we, tx0, ty0, T, STR, PL, nx, ny, flush;
    int accumulate;      // flush 3: add to the grid instead of overwriting it
};

// Flush 3 ("owner tiles"): a work item is an output tile and its list holds every group whose
// footprint reaches the tile, from the tile itself and its neighbours. The wave's LDS tile
// then spans the output tile with a margin of 2h cells (R3 = T + 4h rows), so that every
// such footprint lies inside it, and only the T x T output cells are written, once, straight
// to the grid: no partial buffer and no merge pass.
__host__ __device__ inline int owner_span(int T, int W) { return T + 2 * (W - 1); }
// plane size of a flush-3 tile (row stride R3), congruent to W (mod 32) like the other
// wave tiles so that the component planes of one lane set fall in distinct banks
__host__ __device__ inline int owner_plane(int T, int W) {
    const int R3 = owner_span(T, W);
    int p = R3 * R3;
    while ((p - W) % 32 != 0) p++;
    return p;
}

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

// The NC = 2 * npol components of one cell of a partial tile (cell-major layout, 8 * NC-byte
// aligned) as one or two vector accesses.
template <int NC>
__device__ inline void store_cell(float *dst, const float (&v)[NC]) {
    if constexpr (NC == 2) {
        *(float2 *)dst = make_float2(v[0], v[1]);
    } else {
#pragma unroll
        for (int q = 0; q < NC; q += 4) *(float4 *)(dst + q) = make_float4(v[q], v[q + 1], v[q + 2], v[q + 3]);
    }
}
template <int NC>
__device__ inline void add_cell(const float *src, float (&acc)[NC]) {
    if constexpr (NC == 2) {
        const float2 a = *(const float2 *)src;
        acc[0] += a.x;
        acc[1] += a.y;
    } else {
#pragma unroll
        for (int q = 0; q < NC; q += 4) {
            const float4 a = *(const float4 *)(src + q);
            acc[q] += a.x;
            acc[q + 1] += a.y;
            acc[q + 2] += a.z;
            acc[q + 3] += a.w;
        }
    }
}

// Per-wave staging area of the wave-tile gridder: 32 groups at a time, each as its 2 * npol
// visibility components (slots 0..7) and its column-tap row T[px][0..7] (slots 8..15), at a
// stride of 20 floats: the 16-byte stores of 8 consecutive groups then cover all 32 banks
// once (a stride of 16 would put every other group on the same 4 banks).
constexpr int kStageGroups = 32;
constexpr int kStageStride = 20;
constexpr int kStageFloats = kStageGroups * kStageStride;

// LDS floats per wave of the wave-tile gridder: the staging area, then the tile (NC planes
// of PL floats), rounded so that every wave's staging area stays 16-byte aligned.
__host__ __device__ inline int wavetile_per_wave(int nc, int pl) { return kStageFloats + ((nc * pl + 3) & ~3); }

// Writes a wave's finished private tile out (flush 1: atomic adds into the grid, 2: the
// item's partial slice, cell-major; 3: the owner tile's T x T cells, once).
template <int NPOL, int W>
__device__ inline void wavetile_flush(const ItemCtx &c, int lane) {
    constexpr int NC = 2 * NPOL;
    const int h = (W - 1) / 2, R = c.T + W - 1, STR = c.STR, PL = c.PL;
    const int tx0 = c.tx0, ty0 = c.ty0;
    float *tile = c.tile;
    (void)STR;
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
    } else if (c.flush == 3) {
        // the output tile's T x T cells at LDS offset (2h, 2h), each written once
        const int T = c.T, m = 2 * h;
        for (int idx = lane; idx < T * T; idx += 64) {
            const int r = idx / T, col = idx - r * T;
            const int gy = ty0 + r, gx = tx0 + col;
            if (gy >= c.ny || gx >= c.nx) continue;
            const int o = (r + m) * STR + col + m;
#pragma unroll
            for (int p = 0; p < NPOL; p++) {
                float2 v = make_float2(tile[(2 * p) * PL + o], tile[(2 * p + 1) * PL + o]);
                float2 *dst = c.grid + ((int64_t)p * c.ny + gy) * c.nx + gx;
                if (c.accumulate) {
                    const float2 old = *dst;
                    v.x += old.x;
                    v.y += old.y;
                }
                *dst = v;
            }
        }
    } else if (c.flush == 2) {
        // the item's slice of the partial buffer: cell-major, the NC components of a cell
        // contiguous
        float *out = c.partial;
        for (int idx = lane; idx < R * R; idx += 64) {
            const int r = idx / R, col = idx - r * R;
            float v[NC];
#pragma unroll
            for (int q = 0; q < NC; q++) v[q] = tile[q * PL + r * STR + col];
            store_cell<NC>(out + (int64_t)idx * NC, v);
        }
    }
}

// Grids work item c with this wavefront (lanes as in variant 2) into its private tile and
// writes the tile out (flush 1: atomic adds into the grid, 2: the item's partial slice; 0:
// the tile stays in LDS for the caller). The tile must be zero on entry.
//
// The groups of an item arrive sorted by centre cell and, within a cell, by the row
// sub-position py. The separable tap factorises the work: for a run of groups with the same
// (cell, py), lane (component, column t) first sums T[px][t] * V over the run (one FMA per
// group), and only at the end of the run multiplies that sum into its row accumulators with
// the run's row taps T[py][s]. The row accumulators go to the LDS tile when the cell
// changes. A group costs one FMA instead of W + 1; a run of equal (cell, py) costs W more.
// Both operands of the per-group FMA come from the staging area at fixed offsets, eight
// groups per LDS round trip, so the loop has no per-group address arithmetic.
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
    const float *vbase = sv + cc;     // staged group jl's component: vbase[jl * kStageStride]
    const float *tbase = sv + 8 + t;  // and its column tap T[px][t]
    float acc[NR], ty[NR];
#pragma unroll
    for (int k = 0; k < NR; k++) {
        acc[k] = 0.0f;
        ty[k] = 0.0f;
    }
    float asum = 0.0f;
    int cur = -1;     // current cell (offset in the tile), -1 before the first group
    int curkey = -1;  // current (cell, py) key

    // Ends the current (cell, py) run and starts the one of code qj (a new cell if newcell).
    auto start_run = [&](uint32_t qj, bool newcell) {
#pragma unroll
        for (int k = 0; k < NR; k++) acc[k] = fmaf(ty[k], asum, acc[k]);
        asum = 0.0f;
        if (newcell) {
            if (cur >= 0 && active) wave_tile_add<NR, NSG, W>(tile + cur + loff, STR, sg, acc);
#pragma unroll
            for (int k = 0; k < NR; k++) acc[k] = 0.0f;
            cur = (int)(qj & 0xFFFFu);
        }
        curkey = (int)(qj & 0xFF00FFFFu);
        const int ty8 = (int)(qj >> 24);
        if constexpr (NSG == 1) {
            // every lane needs the whole row: scalar loads from the kernel-argument copy of
            // the table (an LDS broadcast would cost the LDS a full wave of reads)
#pragma unroll
            for (int k = 0; k < NR; k++) ty[k] = c.tapk[ty8 + k];
        } else {
#pragma unroll
            for (int k = 0; k < NR; k++) {
                const int sr = sg + NSG * k;
                ty[k] = ltab[ty8 + (sr < W ? sr : 0)];
            }
        }
    };

    // Software pipeline over batches of 64 groups: lane j holds group j's code and
    // visibilities; the next batch's codes and visibilities and the permutation two batches
    // ahead are in flight while a batch is accumulated.
    uint32_t gA = (wb + lane < we) ? c.perm[wb + lane] : 0u;
    uint32_t gB = (wb + 64 + lane < we) ? c.perm[wb + 64 + lane] : 0u;
    uint32_t qn = (wb + lane < we) ? c.scode[wb + lane] : 0u;
    float2 vn[NPOL];
    if (wb + lane < we) core_fetch<NPOL>(c, wb + lane, gA, vn);

    for (int base = wb; base < we; base += 64) {
        const int cnt = (we - base) < 64 ? (we - base) : 64;
        const uint32_t qcur = qn;
        float2 vc[NPOL];
#pragma unroll
        for (int p = 0; p < NPOL; p++) vc[p] = vn[p];
        if (base + 64 + lane < we) {
            core_fetch<NPOL>(c, base + 64 + lane, gB, vn);
            qn = c.scode[base + 64 + lane];
        }
        gB = (base + 128 + lane < we) ? c.perm[base + 128 + lane] : 0u;
        // Run boundaries: lane j flags whether group j starts a new (cell, py) run and
        // whether it starts a new cell.
        const int cellj = (int)(qcur & 0xFFFFu);
        const int keyj = (int)(qcur & 0xFF00FFFFu);
        int prevc = __shfl_up(cellj, 1, 64);
        int prevk = __shfl_up(keyj, 1, 64);
        if (lane == 0) {
            prevc = cur;
            prevk = curkey;
        }
        const uint64_t kstarts = __ballot(lane < cnt && keyj != prevk);
        const uint64_t cstarts = __ballot(lane < cnt && cellj != prevc);
        for (int h0 = 0; h0 < cnt; h0 += kStageGroups) {
            // stage groups [h0, h0 + 32): visibilities and column-tap rows; positions past
            // the item's end get zeros, so that whole blocks of 8 can be accumulated
            const int jo = lane - h0;
            if (jo >= 0 && jo < kStageGroups) {
                float *dst = sv + jo * kStageStride;
                const bool live = lane < cnt;
                if constexpr (NPOL == 4) {
                    ((float4 *)dst)[0] = live ? make_float4(vc[0].x, vc[0].y, vc[1].x, vc[1].y) : make_float4(0.f, 0.f, 0.f, 0.f);
                    ((float4 *)dst)[1] = live ? make_float4(vc[2].x, vc[2].y, vc[3].x, vc[3].y) : make_float4(0.f, 0.f, 0.f, 0.f);
                } else if constexpr (NPOL == 2) {
                    ((float4 *)dst)[0] = live ? make_float4(vc[0].x, vc[0].y, vc[1].x, vc[1].y) : make_float4(0.f, 0.f, 0.f, 0.f);
                } else {
                    ((float2 *)dst)[0] = live ? vc[0] : make_float2(0.f, 0.f);
                }
                const float4 *row = (const float4 *)(ltab + (live ? ((qcur >> 16) & 0xFFu) : 0u));
                ((float4 *)(dst + 8))[0] = live ? row[0] : make_float4(0.f, 0.f, 0.f, 0.f);
                ((float4 *)(dst + 8))[1] = live ? row[1] : make_float4(0.f, 0.f, 0.f, 0.f);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int hcnt = (cnt - h0) < kStageGroups ? (cnt - h0) : kStageGroups;
            for (int jb = 0; jb < hcnt; jb += 8) {
                float v8[8], t8[8];
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    v8[u] = vbase[(jb + u) * kStageStride];
                    t8[u] = tbase[(jb + u) * kStageStride];
                }
                const int j0 = h0 + jb;
                const uint32_t ks = (uint32_t)(kstarts >> j0) & 0xFFu;  // run starts in this block
                const uint32_t cs = (uint32_t)(cstarts >> j0) & 0xFFu;  // cell starts
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    if ((ks >> u) & 1u)
                        start_run((uint32_t)__builtin_amdgcn_readlane((int)qcur, j0 + u), (cs >> u) & 1u);
                    asum = fmaf(t8[u], v8[u], asum);
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
    start_run(0u, false);  // close the last run (the new run is never used)
    if (cur >= 0 && active) wave_tile_add<NR, NSG, W>(tile + cur + loff, STR, sg, acc);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    wavetile_flush<NPOL, W>(c, lane);
}

// Variant 6 ("block runs"): the work list of variant 4 with every (cell, py) run of a work
// item padded, in the plan, to a multiple of kRunBlock entries (dummies have group index
// kDummyGroup and their run's code, and are staged as zero visibilities). Every block of
// kRunBlock consecutive entries then belongs to one run: a block costs one run-start test,
// one 16-byte LDS read of its visibility components and one of its column taps per lane, and
// kRunBlock FMAs, with no per-group branch. The staging area is component-major: a row of
// kBlockStageStride floats per visibility component and per column tap, 32 entries wide.
// On the MWA-scale workload (runs of 4.9 groups on average, a quarter of them single) the
// padding adds 38 % entries and the launch takes 0.72 ms against variant 4's 0.67 ms, so it
// is not the default.
constexpr int kRunBlock = 4;
constexpr uint32_t kDummyGroup = 0xFFFFFFFFu;
constexpr int kBlockStageStride = 36;  // rows 36 floats apart: 8 rows' 16-byte reads hit distinct banks
__host__ __device__ inline int blocktile_stage_floats(int nc) { return (nc + 8) * kBlockStageStride; }
__host__ __device__ inline int blocktile_per_wave(int nc, int pl) {
    return blocktile_stage_floats(nc) + ((nc * pl + 3) & ~3);
}

template <int NPOL, int W>
__device__ inline void blocktile_item(const ItemCtx &c, int lane) {
    constexpr int NC = 2 * NPOL;
    constexpr int NSG = 8 / NC;
    constexpr int NR = (W + NSG - 1) / NSG;
    constexpr int SS = kBlockStageStride;
    const int STR = c.STR, PL = c.PL;
    float *tile = c.tile, *sv = c.sv;
    const float *ltab = c.ltab;
    const int wb = c.wb, we = c.we;
    const int t = lane % W;
    const int cc = (lane / W) % NC;
    const int sg = lane / (W * NC);
    const bool active = lane < W * NC * NSG;
    const int loff = active ? cc * PL + sg * STR + t : 0;
    const float *vrow = sv + cc * SS;          // component cc of the staged entries
    const float *trow = sv + (NC + t) * SS;    // column tap T[px][t] of the staged entries
    float acc[NR], ty[NR];
#pragma unroll
    for (int k = 0; k < NR; k++) {
        acc[k] = 0.0f;
        ty[k] = 0.0f;
    }
    float asum = 0.0f;
    int cur = -1, curkey = -1;
    auto start_run = [&](uint32_t qj, bool newcell) {
#pragma unroll
        for (int k = 0; k < NR; k++) acc[k] = fmaf(ty[k], asum, acc[k]);
        asum = 0.0f;
        if (newcell) {
            if (cur >= 0 && active) wave_tile_add<NR, NSG, W>(tile + cur + loff, STR, sg, acc);
#pragma unroll
            for (int k = 0; k < NR; k++) acc[k] = 0.0f;
            cur = (int)(qj & 0xFFFFu);
        }
        curkey = (int)(qj & 0xFF00FFFFu);
        const int ty8 = (int)(qj >> 24);
        if constexpr (NSG == 1) {
#pragma unroll
            for (int k = 0; k < NR; k++) ty[k] = c.tapk[ty8 + k];
        } else {
#pragma unroll
            for (int k = 0; k < NR; k++) {
                const int sr = sg + NSG * k;
                ty[k] = ltab[ty8 + (sr < W ? sr : 0)];
            }
        }
    };
    // lane j holds entry j of the batch: its code and visibilities (zero for a dummy); the
    // next batch's are in flight while one is accumulated, the permutation two batches ahead
    uint32_t gA = (wb + lane < we) ? c.perm[wb + lane] : kDummyGroup;
    uint32_t gB = (wb + 64 + lane < we) ? c.perm[wb + 64 + lane] : kDummyGroup;
    uint32_t qn = (wb + lane < we) ? c.scode[wb + lane] : 0u;
    float2 vn[NPOL];
#pragma unroll
    for (int p = 0; p < NPOL; p++) vn[p] = make_float2(0.f, 0.f);
    if (gA != kDummyGroup) core_fetch<NPOL>(c, wb + lane, gA, vn);
    for (int base = wb; base < we; base += 64) {
        const int cnt = (we - base) < 64 ? (we - base) : 64;  // a multiple of kRunBlock
        const uint32_t qcur = qn;
        float2 vc[NPOL];
#pragma unroll
        for (int p = 0; p < NPOL; p++) {
            vc[p] = vn[p];
            vn[p] = make_float2(0.f, 0.f);
        }
        if (base + 64 + lane < we) {
            if (gB != kDummyGroup) core_fetch<NPOL>(c, base + 64 + lane, gB, vn);
            qn = c.scode[base + 64 + lane];
        }
        gB = (base + 128 + lane < we) ? c.perm[base + 128 + lane] : kDummyGroup;
        const int cellj = (int)(qcur & 0xFFFFu);
        const int keyj = (int)(qcur & 0xFF00FFFFu);
        int prevc = __shfl_up(cellj, 1, 64);
        int prevk = __shfl_up(keyj, 1, 64);
        if (lane == 0) {
            prevc = cur;
            prevk = curkey;
        }
        // run and cell starts fall on block boundaries only
        const uint64_t kstarts = __ballot(lane < cnt && keyj != prevk);
        const uint64_t cstarts = __ballot(lane < cnt && cellj != prevc);
        for (int h0 = 0; h0 < cnt; h0 += 32) {
            // stage entries [h0, h0 + 32): components and column-tap rows, component-major
            const int jo = lane - h0;
            if (jo >= 0 && jo < 32) {
                const bool live = lane < cnt;
#pragma unroll
                for (int p = 0; p < NPOL; p++) {
                    sv[(2 * p) * SS + jo] = live ? vc[p].x : 0.0f;
                    sv[(2 * p + 1) * SS + jo] = live ? vc[p].y : 0.0f;
                }
                const float4 *row = (const float4 *)(ltab + (live ? ((qcur >> 16) & 0xFFu) : 0u));
                const float4 r0 = row[0], r1 = row[1];
                float *tr = sv + NC * SS + jo;
                tr[0 * SS] = r0.x;
                tr[1 * SS] = r0.y;
                tr[2 * SS] = r0.z;
                tr[3 * SS] = r0.w;
                tr[4 * SS] = r1.x;
                tr[5 * SS] = r1.y;
                tr[6 * SS] = r1.z;
                tr[7 * SS] = r1.w;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int hcnt = (cnt - h0) < 32 ? (cnt - h0) : 32;  // a multiple of kRunBlock
            const uint64_t ksh = kstarts >> h0, csh = cstarts >> h0;
#pragma unroll
            for (int jb = 0; jb < 32; jb += kRunBlock) {
                if (jb >= hcnt) break;
                const float4 v4 = *(const float4 *)(vrow + jb);
                const float4 t4 = *(const float4 *)(trow + jb);
                if ((ksh >> jb) & 1u)
                    start_run((uint32_t)__builtin_amdgcn_readlane((int)qcur, h0 + jb), (csh >> jb) & 1u);
                asum = fmaf(t4.x, v4.x, asum);
                asum = fmaf(t4.y, v4.y, asum);
                asum = fmaf(t4.z, v4.z, asum);
                asum = fmaf(t4.w, v4.w, asum);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
    start_run(0u, false);  // close the last run
    if (cur >= 0 && active) wave_tile_add<NR, NSG, W>(tile + cur + loff, STR, sg, acc);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    wavetile_flush<NPOL, W>(c, lane);
}

// The merge pass over blocks of kMergeB x kMergeB cells, one cell per thread. Every cell is
// the sum over the partial tiles of the work items whose haloed tile covers it, in a fixed
// order (tile row, tile column, then the tile's work items), so the result is
// bit-reproducible. The work-item ranges of the tiles that can cover a block are staged in
// LDS first: a span of 16 + 2h cells meets at most floor((15 + 2h) / T) + 2 tiles per axis,
// which is 5 for T >= 8 and h <= 7 (W <= 15) (a kMergeTiles table). Only blocks that some
// work item reaches are listed for the merge; the plan lists the others apart and a plain
// fill writes their zeros.

struct MergeBounds {
    int tx_lo, ty_lo, ntxb, ntyb;
};

__device__ inline MergeBounds merge_bounds(int x0, int y0, int h, int lgT, int ntx, int nty) {
    MergeBounds m;
    m.tx_lo = max(0, x0 - h) >> lgT;
    m.ty_lo = max(0, y0 - h) >> lgT;
    m.ntxb = min(ntx - 1, (x0 + kMergeB - 1 + h) >> lgT) - m.tx_lo + 1;
    m.ntyb = min(nty - 1, (y0 + kMergeB - 1 + h) >> lgT) - m.ty_lo + 1;
    return m;
}

// Entry e of block (x0, y0)'s tile-range table.
// (fid: the tile's first work item, or -1 for a tile with none)
__device__ inline void merge_stage(const int32_t *tile_work, const int32_t *work_ids, int ntx, const MergeBounds &m,
                                   int e, int2 *rng, int *fid) {
    if (e < m.ntxb * m.ntyb) {
        const int t = (m.ty_lo + e / m.ntxb) * ntx + m.tx_lo + e % m.ntxb;
        const int2 rg = make_int2(tile_work[t], tile_work[t + 1]);
        rng[e] = rg;
        fid[e] = rg.y > rg.x ? work_ids[rg.x] : -1;
    }
}

template <int NPOL>
__device__ inline void merge_cell(float2 *grid, const float *partial, const int32_t *work_ids, int nx, int ny,
                                  int lgT, int W, int accumulate, const MergeBounds &m, const int2 *rng,
                                  const int *fid, int x, int y) {
    constexpr int NC = 2 * NPOL;
    const int T = 1 << lgT, h = (W - 1) / 2, R = T + W - 1;
    if (x >= nx || y >= ny) return;
    const int txc = x >> lgT, tyc = y >> lgT;
    float acc[NC];
#pragma unroll
    for (int q = 0; q < NC; q++) acc[q] = 0.0f;
    if constexpr (NC <= 4) {
        // few components: load the first work item's value of each of the <= 3 x 3 covering
        // tiles with all loads in flight together, then add them, and any further items of a
        // split tile, in the fixed order (tile row, tile column, then the tile's items)
        float first[9][NC];
        int ent[9], off[9];
#pragma unroll
        for (int t = 0; t < 9; t++) {
            const int tty = tyc + t / 3 - 1, ttx = txc + t % 3 - 1;
            const int r = y - (tty * T - h), c = x - (ttx * T - h);
            const bool ok = tty >= m.ty_lo && tty < m.ty_lo + m.ntyb && r >= 0 && r < R && ttx >= m.tx_lo &&
                            ttx < m.tx_lo + m.ntxb && c >= 0 && c < R;
            ent[t] = ok ? (tty - m.ty_lo) * m.ntxb + (ttx - m.tx_lo) : -1;
            off[t] = r * R + c;
            const int f = ok ? fid[ent[t]] : -1;
#pragma unroll
            for (int q = 0; q < NC; q++) first[t][q] = 0.0f;
            if (f >= 0) add_cell<NC>(partial + ((int64_t)f * R * R + off[t]) * NC, first[t]);
        }
#pragma unroll
        for (int t = 0; t < 9; t++) {
            if (ent[t] < 0) continue;
            const int2 rg = rng[ent[t]];
            if (rg.y <= rg.x) continue;
#pragma unroll
            for (int q = 0; q < NC; q++) acc[q] += first[t][q];
            for (int k = rg.x + 1; k < rg.y; k++)
                add_cell<NC>(partial + ((int64_t)work_ids[k] * R * R + off[t]) * NC, acc);
        }
    } else if (2 * h <= T) {
        // 8 components, at most two covering tiles per axis (the halo is at most half a
        // tile): the rows tyc + dy0 and tyc + dy0 + 1 and the columns likewise, with the four
        // first-item loads in flight together, then the same order as below
        float first[4][NC];
        int ent[4], off[4];
        const int dy0 = (y & (T - 1)) < h ? -1 : 0, dx0 = (x & (T - 1)) < h ? -1 : 0;
#pragma unroll
        for (int t = 0; t < 4; t++) {
            const int tty = tyc + dy0 + (t >> 1), ttx = txc + dx0 + (t & 1);
            const int r = y - (tty * T - h), c = x - (ttx * T - h);
            const bool ok = tty >= m.ty_lo && tty < m.ty_lo + m.ntyb && r >= 0 && r < R && ttx >= m.tx_lo &&
                            ttx < m.tx_lo + m.ntxb && c >= 0 && c < R;
            ent[t] = ok ? (tty - m.ty_lo) * m.ntxb + (ttx - m.tx_lo) : -1;
            off[t] = r * R + c;
            const int f = ok ? fid[ent[t]] : -1;
#pragma unroll
            for (int q = 0; q < NC; q++) first[t][q] = 0.0f;
            if (f >= 0) add_cell<NC>(partial + ((int64_t)f * R * R + off[t]) * NC, first[t]);
        }
#pragma unroll
        for (int t = 0; t < 4; t++) {
            if (ent[t] < 0) continue;
            const int2 rg = rng[ent[t]];
            if (rg.y <= rg.x) continue;
#pragma unroll
            for (int q = 0; q < NC; q++) acc[q] += first[t][q];
            for (int k = rg.x + 1; k < rg.y; k++)
                add_cell<NC>(partial + ((int64_t)work_ids[k] * R * R + off[t]) * NC, acc);
        }
    } else {
        // 8 components and wider halos: the same order, one tile at a time (holding nine
        // tiles' values would cost more registers than the overlap gains)
        for (int dy = -1; dy <= 1; dy++) {
            const int tty = tyc + dy;
            if (tty < m.ty_lo || tty >= m.ty_lo + m.ntyb) continue;
            const int r = y - (tty * T - h);
            if (r < 0 || r >= R) continue;
            for (int dx = -1; dx <= 1; dx++) {
                const int ttx = txc + dx;
                if (ttx < m.tx_lo || ttx >= m.tx_lo + m.ntxb) continue;
                const int c = x - (ttx * T - h);
                if (c < 0 || c >= R) continue;
                const int2 rg = rng[(tty - m.ty_lo) * m.ntxb + (ttx - m.tx_lo)];
                for (int k = rg.x; k < rg.y; k++)
                    add_cell<NC>(partial + ((int64_t)work_ids[k] * R * R + r * R + c) * NC, acc);
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

// Zeros of one merge block (the NPOL planes of its cells), kMergeB^2 threads.
template <int NPOL>
__device__ inline void zero_block(float2 *grid, int nx, int ny, int x0, int y0) {
    const int x = x0 + (threadIdx.x & (kMergeB - 1)), y = y0 + threadIdx.x / kMergeB;
    if (x >= nx || y >= ny) return;
#pragma unroll
    for (int p = 0; p < NPOL; p++) grid[((int64_t)p * ny + y) * nx + x] = make_float2(0.f, 0.f);
}

// Zeros of one T x T output tile (origin x0, y0) in the NPOL planes of a grid, written by
// nl lanes (lane l) with 16-byte stores where the row allows (T >= 2, x0 even).
template <int NPOL>
__device__ inline void zero_tile(float2 *grid, int nx, int ny, int x0, int y0, int T, int l, int nl) {
    const int half = T / 2;  // float4 (two cells) per row position
    const bool vec = (nx % 2) == 0 && ((uintptr_t)grid & 15u) == 0;
    for (int idx = l; idx < T * half; idx += nl) {
        const int r = idx / half, c2 = idx - r * half;
        const int gy = y0 + r, gx = x0 + 2 * c2;
        if (gy >= ny || gx >= nx) continue;
#pragma unroll
        for (int p = 0; p < NPOL; p++) {
            float2 *dst = grid + ((int64_t)p * ny + gy) * nx + gx;
            if (vec && gx + 1 < nx) {
                *(float4 *)dst = make_float4(0.f, 0.f, 0.f, 0.f);
            } else {
                dst[0] = make_float2(0.f, 0.f);
                if (gx + 1 < nx) dst[1] = make_float2(0.f, 0.f);
            }
        }
    }
}

} // namespace mwg
