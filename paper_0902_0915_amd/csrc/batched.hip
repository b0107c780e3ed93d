// Batched form of a multi-instance plan: many uneven gridding instances (snapshots,
// channels) in one launch sequence, replayed from a captured hipGraph.
//
// Gridding: one launch over the (instance, work item) pairs of all instances, one pair per
// wavefront, in instance order; each item is gridded with the wave-tile body shared with
// the single-instance gridder (gridder_core.h). Then one merge launch over the cell blocks
// of every instance's grid that some work item reaches, and one launch that writes zeros to
// the other blocks, both over (instance, block) lists built with the plan. Degridding: one launch over all instances' work items
// with the shared degrid body (degrid_core.h), after one prologue launch that zeroes the
// outputs of dropped groups and the gain gradients.
//
// Per-call pointers (visibilities, gains, grids) live in a device descriptor table that is
// refreshed by an asynchronous copy on the caller's stream before each graph replay, so the
// captured graph stays valid when the caller's buffers change. The graphs are captured on a
// stream owned by the plan and replayed on the caller's stream.
#include "internal.h"
#include "degrid_core.h"
#include "gridder_core.h"

#include <algorithm>
#include <cstdlib>
#include <cstring>

namespace mwg {

size_t wavetiles_lds(int npol, int T, int W, int O, int waves);
size_t owner_lds(int npol, int T, int W, int O, int waves);
Status launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);
Status ensure_partial(Instance &I, hipStream_t s);

namespace {

// Most groups an output tile may receive for an instance of a batch to take the owner-tile
// flush (one wave grids the whole list).
constexpr int64_t kOwnerCap = 4096;

struct BatchDesc {
    // refreshed per call
    const float2 *vis, *gains, *vis_in;
    float2 *grid, *vis_out, *grad_gains;
    int32_t accumulate, pad0;
    // fixed at plan time
    const uint32_t *perm, *spos, *scode, *sant, *dropped;
    const float *sw, *tab;
    const WorkItem *work;
    float *partial;
    const int32_t *tile_work, *work_ids;
    const int32_t *mblocks; // merge blocks some work item reaches, then those none reaches
    int32_t nx, ny, ntx, nty, nwork, nant, ndropped, n_mblocks;
    // flush 3 (owner tiles): the instance's work items are output tiles over its pair lists
    int32_t flush;
    int32_t item0;  // index of the instance's first gridder record in the batch
    const WorkItem *owork;
    const uint32_t *pperm, *pcode, *psant;
    const float *psw;
};

struct BatchItem {
    int32_t inst, item;
};

// One gridder work item of the batch, self-contained so that a wave needs one record load
// before it can start on the item's groups: the instance, the tile (index in the instance's
// tile grid), the group range and the arrays it indexes (sorted or per-pair).
struct GridItem {
    int32_t inst, tile, begin, end;
    const uint32_t *perm, *code;
};

struct Batch {
    int ninst = 0, npol = 1, W = 7, O = 8, T = 8, waves = 8, STR = 0, PL = 0, nitems = 0;
    int STR3 = 0, PL3 = 0, per_wave = 0;  // flush-3 LDS tile; LDS floats per wave (either form)
    int64_t ztiles = 0;                   // output tiles of flush-3 instances written as zeros
    int dthreads = 256;  // threads per degridder workgroup
    int grid_blocks = 0;     // gridder workgroups (waves of them, one work item per wave)
    int64_t merge_blocks = 0, zero_blocks = 0, prologue_n = 0;
    int ant_in_lds = 0;
    size_t grid_lds = 0, degrid_lds = 0;
    DevArena arena;
    BatchDesc *d_desc = nullptr, *h_desc = nullptr; // h_desc: pinned host memory
    hipEvent_t desc_ev = nullptr;
    bool desc_pending = false;
    GridItem *d_items = nullptr;    // gridder items (owner tiles for flush-3 instances)
    hipStream_t side = nullptr;     // second branch of the gridding sequence (zero fills)
    hipEvent_t fork = nullptr, join = nullptr;
    BatchItem *d_ditems = nullptr;  // degridder items (every instance's source-tile items)
    int nditems = 0;
    int64_t *d_pro_start = nullptr;
    int2 *d_mpairs = nullptr; // (instance, block) of every merge block, then of every zero block
    int2 *d_ztiles = nullptr; // (instance, output tile) of every zero tile of flush-3 instances
    const float *tab8 = nullptr;
    float tapk[16 * 8] = {0};
    hipStream_t cap = nullptr;
    hipGraphExec_t x_grid = nullptr, x_degrid = nullptr;
    bool use_graph = true;
};

struct BatchGridArgs {
    const BatchDesc *desc;
    const GridItem *items;
    const float *tab8;
    int nitems, O, T, STR, PL, STR3, PL3, per_wave;
    float tapk[16 * 8];
};

// Wave-uniform copies of values loaded from the descriptor table. Without them the
// compiler may keep such values in VGPRs, and every loop of the item body then becomes an
// exec-masked divergent loop.
__device__ inline int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

template <class T>
__device__ inline T *uni(T *p) {
    const uint64_t u = (uint64_t)p;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
    return (T *)(((uint64_t)hi << 32) | lo);
}

template <int NPOL, int W>
__global__ __launch_bounds__(1024) void k_grid_batched(BatchGridArgs a) {
    constexpr int NC = 2 * NPOL;
    extern __shared__ __align__(16) float smem[];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int ntab = a.O * 8;
    float *ltab = smem;
    // the item's record is loaded before the tap-table barrier, so that the two loads overlap
    const int w = blockIdx.x * (int)(blockDim.x >> 6) + wave;
    const GridItem it = a.items[w < a.nitems ? w : 0];
    for (int i = tid; i < ntab; i += blockDim.x) ltab[i] = a.tab8[i];
    __syncthreads();
    if (w >= a.nitems) return;
    const int R = a.T + W - 1;
    float *stage = smem + ntab + wave * a.per_wave;
    const int inst = uni(it.inst), wtile = uni(it.tile);
    const BatchDesc &d = a.desc[inst];
    const bool owner = uni(d.flush) == 3;
    const int ntx = uni(d.ntx);
    const int PL = owner ? a.PL3 : a.PL;
    float *tile = stage + kStageFloats;
    for (int i = 4 * lane; i < NC * PL; i += 256) *(float4 *)(tile + i) = make_float4(0.f, 0.f, 0.f, 0.f);
    ItemCtx c;
    c.tile = tile;
    c.sv = stage;
    c.vis = uni(d.vis);
    c.gains = uni(d.gains);
    c.perm = uni(it.perm);
    c.scode = uni(it.code);
    c.sant = uni(owner ? d.psant : d.sant);
    c.sw = uni(owner ? d.psw : d.sw);
    c.tapk = a.tapk;
    c.ltab = ltab;
    c.grid = uni(d.grid);
    // flush 2: the item's partial slice (items of an instance are numbered by its work list,
    // the record's position within the instance's contiguous run of records)
    c.partial = owner ? nullptr : uni(d.partial) + (int64_t)(w - uni(d.item0)) * NC * R * R;
    c.wb = uni(it.begin);
    c.we = uni(it.end);
    c.tx0 = (wtile % ntx) * a.T;
    c.ty0 = (wtile / ntx) * a.T;
    c.T = a.T;
    c.STR = owner ? a.STR3 : a.STR;
    c.PL = PL;
    c.nx = uni(d.nx);
    c.ny = uni(d.ny);
    c.flush = owner ? 3 : 2;
    c.accumulate = uni(d.accumulate);
    wavetile_item<NPOL, W>(c, lane);
}

__device__ inline int find_inst(const int64_t *start, int n, int64_t b) {
    int lo = 0, hi = n - 1; // largest i with start[i] <= b
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// The merge pass over every instance's listed blocks that some work item reaches, one
// (instance, block) pair of the concatenated list per workgroup.
template <int NPOL>
__global__ __launch_bounds__(kMergeB * kMergeB) void k_merge_batched(const BatchDesc *desc, const int2 *pairs,
                                                                     int lgT, int W) {
    __shared__ int2 rng[kMergeTiles];
    __shared__ int fid[kMergeTiles];
    const int h = (W - 1) / 2, tid = threadIdx.x;
    const int2 pr = pairs[blockIdx.x];
    const BatchDesc &d = desc[pr.x];
    const int bpr = (d.nx + kMergeB - 1) / kMergeB;
    const int by = pr.y / bpr, bx = pr.y - by * bpr;
    const int x0 = bx * kMergeB, y0 = by * kMergeB;
    const MergeBounds m = merge_bounds(x0, y0, h, lgT, d.ntx, d.nty);
    if (tid < 32) merge_stage(d.tile_work, d.work_ids, d.ntx, m, tid, rng, fid);
    __syncthreads();
    merge_cell<NPOL>(d.grid, d.partial, d.work_ids, d.nx, d.ny, lgT, W, d.accumulate, m, rng, fid,
                     x0 + (tid & (kMergeB - 1)), y0 + tid / kMergeB);
}

// Zeros of every instance's listed blocks that no work item reaches (nothing when
// accumulating).
template <int NPOL>
__global__ __launch_bounds__(kMergeB * kMergeB) void k_zero_batched(const BatchDesc *desc, const int2 *pairs) {
    const int2 pr = pairs[blockIdx.x];
    const BatchDesc &d = desc[pr.x];
    if (d.accumulate) return;
    const int bpr = (d.nx + kMergeB - 1) / kMergeB;
    const int by = pr.y / bpr, bx = pr.y - by * bpr;
    zero_block<NPOL>(d.grid, d.nx, d.ny, bx * kMergeB, by * kMergeB);
}

// Zeros of the output tiles of flush-3 instances that no footprint reaches (nothing when
// accumulating), one tile per wave.
template <int NPOL>
__global__ __launch_bounds__(256) void k_zero_tiles_batched(const BatchDesc *desc, const int2 *pairs, int64_t n,
                                                            int T) {
    const int wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    const int64_t nw = (int64_t)gridDim.x * 4;
    for (int64_t k = (int64_t)blockIdx.x * 4 + wave; k < n; k += nw) {
        const int2 pr = pairs[k];
        const BatchDesc &d = desc[pr.x];
        if (d.accumulate) continue;
        zero_tile<NPOL>(d.grid, d.nx, d.ny, (pr.y % d.ntx) * T, (pr.y / d.ntx) * T, T, lane, 64);
    }
}

// Zeroes the adjoint outputs of dropped groups (entries [0, start[ninst]) of the dropped
// lists) and the gain gradients (the next sum of nant entries).
template <int NPOL>
__global__ void k_degrid_prologue(const BatchDesc *desc, const int64_t *start, int ninst,
                                  int64_t ndrop_total) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= start[2 * ninst]) return;
    if (i < ndrop_total) {
        const int inst = find_inst(start, ninst, i);
        const BatchDesc &d = desc[inst];
        float2 *dst = d.vis_out + (int64_t)d.dropped[i - start[inst]] * NPOL;
#pragma unroll
        for (int p = 0; p < NPOL; p++) dst[p] = make_float2(0.f, 0.f);
    } else {
        const int inst = find_inst(start + ninst, ninst, i);
        const BatchDesc &d = desc[inst];
        if (d.grad_gains) d.grad_gains[i - start[ninst + inst]] = make_float2(0.f, 0.f);
    }
}

template <int NPOL, int WT>
__global__ __launch_bounds__(256) void k_degrid_batched(const BatchDesc *desc, const BatchItem *items,
                                                        int T, int W, int O, int ant_in_lds) {
    extern __shared__ __align__(16) float smem[];
    const BatchItem it = items[blockIdx.x];
    const BatchDesc &d = desc[it.inst];
    DegridArgs a;
    a.grid = d.grid;
    a.gains = d.gains;
    a.vis_in = d.vis_in;
    a.vis_out = d.vis_out;
    a.grad_gains = d.grad_gains;
    a.perm = d.perm;
    a.spos = d.spos;
    a.sant = d.sant;
    a.sw = d.sw;
    a.work = d.work;
    a.tab = d.tab;
    a.nx = d.nx;
    a.ny = d.ny;
    a.T = T;
    a.ntx = d.ntx;
    a.W = W;
    a.O = O;
    a.nant = d.nant;
    a.ant_in_lds = ant_in_lds;
    if constexpr (NPOL == 4 && WT > 0)
        degrid_item_runs<NPOL, WT>(a, d.work[it.item], smem);
    else
        degrid_item<NPOL, WT>(a, d.work[it.item], smem);
}

int plane2(int R, int STR, int W) {
    int p = R * STR;
    while ((p - W) % 32 != 0) p++;
    return p;
}

template <int NPOL>
Status enqueue_grid(Batch &B, hipStream_t s) {
    BatchGridArgs a;
    a.desc = B.d_desc;
    a.items = B.d_items;
    a.tab8 = B.tab8;
    a.nitems = B.nitems;
    a.O = B.O;
    a.T = B.T;
    a.STR = B.STR;
    a.PL = B.PL;
    a.STR3 = B.STR3;
    a.PL3 = B.PL3;
    a.per_wave = B.per_wave;
    std::memcpy(a.tapk, B.tapk, sizeof a.tapk);
    // The zero fills write cells no work item reaches, disjoint from everything the gridder
    // and the merge write: they run on a second branch (a parallel branch of the captured
    // graph), so the bandwidth-bound fill overlaps the latency-bound gridder.
    const bool fork = B.zero_blocks > 0 || B.ztiles > 0;
    if (fork) {
        MWG_HIP(hipEventRecord(B.fork, s));
        MWG_HIP(hipStreamWaitEvent(B.side, B.fork, 0));
        if (B.zero_blocks > 0) {
            hipLaunchKernelGGL(k_zero_batched<NPOL>, dim3((unsigned)B.zero_blocks), dim3(kMergeB * kMergeB), 0,
                               B.side, B.d_desc, (const int2 *)B.d_mpairs + B.merge_blocks);
            MWG_HIP(hipGetLastError());
        }
        if (B.ztiles > 0) {
            const int64_t wg = std::min<int64_t>((B.ztiles + 3) / 4, 4096);
            hipLaunchKernelGGL(k_zero_tiles_batched<NPOL>, dim3((unsigned)wg), dim3(256), 0, B.side, B.d_desc,
                               (const int2 *)B.d_ztiles, B.ztiles, B.T);
            MWG_HIP(hipGetLastError());
        }
        MWG_HIP(hipEventRecord(B.join, B.side));
    }
    const dim3 g(B.grid_blocks), b(64 * B.waves);
    switch (B.W) {
    case 3: hipLaunchKernelGGL((k_grid_batched<NPOL, 3>), g, b, B.grid_lds, s, a); break;
    case 5: hipLaunchKernelGGL((k_grid_batched<NPOL, 5>), g, b, B.grid_lds, s, a); break;
    case 7: hipLaunchKernelGGL((k_grid_batched<NPOL, 7>), g, b, B.grid_lds, s, a); break;
    default: return make_error(MW_ERR_UNSUPPORTED, "batched gridder needs W in {3, 5, 7}");
    }
    MWG_HIP(hipGetLastError());
    if (B.merge_blocks > 0) {
        hipLaunchKernelGGL(k_merge_batched<NPOL>, dim3((unsigned)B.merge_blocks), dim3(kMergeB * kMergeB), 0, s,
                           B.d_desc, (const int2 *)B.d_mpairs, ilog2(B.T), B.W);
        MWG_HIP(hipGetLastError());
    }
    if (fork) MWG_HIP(hipStreamWaitEvent(s, B.join, 0));
    return Status::Ok();
}

template <int NPOL>
Status enqueue_degrid(Batch &B, int64_t ndrop_total, hipStream_t s) {
    if (B.prologue_n > 0) {
        hipLaunchKernelGGL(k_degrid_prologue<NPOL>, dim3((unsigned)((B.prologue_n + 255) / 256)), dim3(256), 0,
                           s, B.d_desc, (const int64_t *)B.d_pro_start, B.ninst, ndrop_total);
        MWG_HIP(hipGetLastError());
    }
    if (B.nditems > 0) {
        const dim3 grid((unsigned)B.nditems), block((unsigned)B.dthreads);
        switch (B.W) {  // the common supports with their taps in registers
        case 3:
            hipLaunchKernelGGL((k_degrid_batched<NPOL, 3>), grid, block, B.degrid_lds, s, B.d_desc, B.d_ditems, B.T,
                               B.W, B.O, B.ant_in_lds);
            break;
        case 5:
            hipLaunchKernelGGL((k_degrid_batched<NPOL, 5>), grid, block, B.degrid_lds, s, B.d_desc, B.d_ditems, B.T,
                               B.W, B.O, B.ant_in_lds);
            break;
        case 7:
            hipLaunchKernelGGL((k_degrid_batched<NPOL, 7>), grid, block, B.degrid_lds, s, B.d_desc, B.d_ditems, B.T,
                               B.W, B.O, B.ant_in_lds);
            break;
        default:
            hipLaunchKernelGGL((k_degrid_batched<NPOL, 0>), grid, block, B.degrid_lds, s, B.d_desc, B.d_ditems, B.T,
                               B.W, B.O, B.ant_in_lds);
            break;
        }
        MWG_HIP(hipGetLastError());
    }
    return Status::Ok();
}

Status enqueue(Batch &B, bool degrid, int64_t ndrop_total, hipStream_t s) {
    switch (B.npol) {
    case 1: return degrid ? enqueue_degrid<1>(B, ndrop_total, s) : enqueue_grid<1>(B, s);
    case 2: return degrid ? enqueue_degrid<2>(B, ndrop_total, s) : enqueue_grid<2>(B, s);
    case 4: return degrid ? enqueue_degrid<4>(B, ndrop_total, s) : enqueue_grid<4>(B, s);
    default: return make_error(MW_ERR_UNSUPPORTED, "npol %d", B.npol);
    }
}

// Captures the grid or degrid sequence on the plan's stream once; later calls replay it.
Status run(Batch &B, bool degrid, int64_t ndrop_total, hipStream_t s) {
    if (!B.use_graph) return enqueue(B, degrid, ndrop_total, s);
    hipGraphExec_t &x = degrid ? B.x_degrid : B.x_grid;
    if (!x) {
        hipGraph_t g = nullptr;
        MWG_HIP(hipStreamBeginCapture(B.cap, hipStreamCaptureModeRelaxed));
        Status st = enqueue(B, degrid, ndrop_total, B.cap);
        hipError_t e = hipStreamEndCapture(B.cap, &g);
        if (!st.ok()) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return make_error(MW_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            x = nullptr;
            return make_error(MW_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
        }
    }
    MWG_HIP(hipGraphLaunch(x, s));
    return Status::Ok();
}

// Writes the per-call fields into the pinned table and copies it to the device on s.
Status refresh_desc(Batch &B, const void *const *vis, const void *const *gains, const void *const *vis_in,
                    void *const *grid, void *const *vis_out, void *const *grad, int accumulate,
                    hipStream_t s) {
    if (B.desc_pending) {
        MWG_HIP(hipEventSynchronize(B.desc_ev)); // the previous copy has read the table
        B.desc_pending = false;
    }
    for (int i = 0; i < B.ninst; i++) {
        BatchDesc &d = B.h_desc[i];
        d.vis = vis ? (const float2 *)vis[i] : nullptr;
        d.gains = gains ? (const float2 *)gains[i] : nullptr;
        d.vis_in = vis_in ? (const float2 *)vis_in[i] : nullptr;
        d.grid = grid ? (float2 *)grid[i] : nullptr;
        d.vis_out = vis_out ? (float2 *)vis_out[i] : nullptr;
        d.grad_gains = grad ? (float2 *)grad[i] : nullptr;
        d.accumulate = accumulate;
    }
    MWG_HIP(hipMemcpyAsync(B.d_desc, B.h_desc, sizeof(BatchDesc) * B.ninst, hipMemcpyHostToDevice, s));
    MWG_HIP(hipEventRecord(B.desc_ev, s));
    B.desc_pending = true;
    return Status::Ok();
}

} // namespace

// The batched form serves plans whose instances share npol, W, O and the wave-tile launch
// (variant 4, merge flush, same tile and waves); other plans run instance by instance.
Status batch_prepare(Plan &P, hipStream_t s) {
    P.batch = nullptr;
    const int n = (int)P.inst.size();
    // Sparse batches (fewer than 64 kept groups per occupied 8 x 8 tile on average) take
    // 16 x 16 tiles: a quarter of the work items, each staging and flushing less halo per
    // group. The batch as a whole still has items enough to fill the chip, which one sparse
    // instance on its own does not, so single-instance plans keep 8 x 8. The choice needs only
    // the occupied-tile counts of the positions pass, so an instance whose schedule was
    // deferred is sorted once, at its final tile.
    std::vector<Launch> Ls((size_t)n);
    {
        bool retile = n >= 2;
        int64_t kept = 0, tiles = 0;
        for (const Instance *I : P.inst) {
            retile = retile && !I->stacks && !I->tile_fixed && I->L.variant == 4 && I->L.flush == 2 &&
                     I->L.tile == 8 && I->L.schedule == 1 &&
                     wavetiles_lds(I->npol, 16, I->W, I->O, I->L.wg_waves) <= 160 * 1024;
            kept += I->nkept;
            tiles += I->ntiles8;
        }
        retile = retile && tiles > 0 && kept < 64 * tiles;
        for (int i = 0; i < n; i++) {
            Ls[(size_t)i] = P.inst[(size_t)i]->L;
            if (retile) Ls[(size_t)i].tile = 16;
        }
    }
    // The batched form serves instances that share npol, W, O and the wave-tile launch.
    bool batchable = n >= 2;
    for (int i = 0; i < n && batchable; i++) {
        const Instance &I = *P.inst[(size_t)i], &I0 = *P.inst[0];
        const Launch &L = Ls[(size_t)i], &L0 = Ls[0];
        batchable = !I.stacks && I.npol == I0.npol && I.W == I0.W && I.O == I0.O && L.variant == 4 &&
                    (L.flush == 2 || L.flush == 3) && L.schedule == 1 && L.tile == L0.tile &&
                    L.wg_waves == L0.wg_waves;
    }
    // Per instance (in parallel for many): the schedule at its final launch, then, in a batch,
    // the owner-tile flush for instances whose output tiles each receive at most kOwnerCap
    // groups (every cell written once, no scratch tiles, no merge; denser ones keep the merge).
    auto prepare = [&](int i, hipStream_t ws) -> Status {
        Instance &I = *P.inst[(size_t)i];
        const Launch &L = Ls[(size_t)i];
        if (!I.scheduled || L.tile != I.L.tile) MWG_TRY(schedule_instance(I, L, ws));
        if (!batchable || I.L.flush != 2 || I.flush_fixed || I.L.tile < I.W - 1 ||
            owner_lds(I.npol, I.L.tile, I.W, I.O, I.L.wg_waves) > 160 * 1024)
            return Status::Ok();
        bool built = false;
        MWG_TRY(build_owner_schedule(I, kOwnerCap, &built, ws));
        if (built) I.L.flush = 3;
        return Status::Ok();
    };
    if (n >= 4) {
        size_t hint = 0;
        for (const Instance *I : P.inst) hint = std::max(hint, plan_tmp_hint(I->ngroups, I->nx, I->ny));
        MWG_TRY(parallel_instances(P.device, n, s, prepare, hint));
    } else {
        for (int i = 0; i < n; i++) MWG_TRY(prepare(i, s));
    }
    if (!batchable) return Status::Ok();
    const Instance &I0 = *P.inst[0];
    Batch *B = new Batch();
    P.batch = B;
    B->ninst = (int)P.inst.size();
    B->npol = I0.npol;
    B->W = I0.W;
    B->O = I0.O;
    B->T = I0.L.tile;
    B->waves = I0.L.wg_waves;
    const int R = B->T + B->W - 1;
    B->STR = R;
    B->PL = plane2(R, R, B->W);
    B->STR3 = owner_span(B->T, B->W);
    B->PL3 = owner_plane(B->T, B->W);
    {
        bool any3 = false;
        for (const Instance *I : P.inst) any3 = any3 || I->L.flush == 3;
        B->per_wave = std::max(wavetile_per_wave(2 * B->npol, B->PL),
                               any3 ? wavetile_per_wave(2 * B->npol, B->PL3) : 0);
    }
    B->tab8 = I0.tab8;
    for (int r = 0; r < I0.O; r++)
        for (int t = 0; t < I0.W; t++) B->tapk[r * 8 + t] = I0.h_tab[(size_t)r * I0.W + t];
    const char *ng = std::getenv("MW_NO_GRAPH");
    B->use_graph = !(ng && ng[0] == '1');
    // descriptors (fixed part)
    std::vector<BatchDesc> desc(B->ninst);
    std::vector<GridItem> items;
    std::vector<BatchItem> ditems;
    std::vector<int64_t> pstart(2 * B->ninst + 1, 0);
    int max_nant = 0;
    for (int i = 0; i < B->ninst; i++) {
        Instance &I = *P.inst[i];
        const bool owner = I.L.flush == 3;
        if (!owner) MWG_TRY(ensure_partial(I, s));
        BatchDesc &d = desc[i];
        std::memset(&d, 0, sizeof d);
        d.perm = I.perm;
        d.spos = I.spos;
        d.scode = I.scode;
        d.sant = I.sant;
        d.dropped = I.dropped;
        d.sw = I.sw;
        d.tab = I.tab;
        d.work = I.work;
        d.partial = I.partial;
        d.tile_work = I.tile_work;
        d.work_ids = I.work_ids;
        d.mblocks = I.mblocks;
        d.n_mblocks = I.n_mblocks;
        d.nx = I.nx;
        d.ny = I.ny;
        d.ntx = I.ntx;
        d.nty = I.nty;
        d.nwork = I.nwork;
        d.nant = I.nant;
        d.ndropped = (int)(I.ngroups - I.nkept);
        d.flush = I.L.flush;
        if (owner) {
            d.owork = I.owork;
            d.pperm = I.pperm;
            d.pcode = I.pcode;
            d.psant = I.psant;
            d.psw = I.psw;
        }
        max_nant = std::max(max_nant, I.nant);
        {
            const std::vector<WorkItem> &wl = owner ? I.h_owork : I.h_work;
            d.item0 = (int32_t)items.size();
            for (const WorkItem &wk : wl)
                items.push_back({i, wk.tile, wk.begin, wk.end, owner ? I.pperm : I.perm, owner ? I.pcode : I.scode});
        }
        for (int w = 0; w < I.nwork; w++) ditems.push_back({i, w});
        pstart[i + 1] = pstart[i] + d.ndropped;
    }
    // second half: gain-gradient entries, numbered after all dropped entries
    for (int i = 0; i < B->ninst; i++) pstart[B->ninst + i + 1] = pstart[B->ninst + i] + desc[i].nant;
    B->prologue_n = pstart[2 * B->ninst];
    // Items stay in instance order (largest first within an instance, as each work list is
    // built): the waves in flight then gather from one or two instances' visibilities at a
    // time, which stay in cache. Interleaving all instances largest-first spreads the random
    // gathers over every instance at once and runs ~4x slower.
    B->nitems = (int)items.size();
    B->nditems = (int)ditems.size();
    {
        int64_t kept = 0;
        for (Instance *I : P.inst) kept += I->nkept;
        B->dthreads = degrid_threads(kept, B->nditems);
    }
    void *p;
    MWG_TRY(B->arena.alloc(&p, sizeof(BatchDesc) * B->ninst));
    B->d_desc = (BatchDesc *)p;
    if (hipHostMalloc((void **)&B->h_desc, sizeof(BatchDesc) * B->ninst, hipHostMallocDefault) != hipSuccess) {
        B->h_desc = nullptr;
        return make_error(MW_ERR_ALLOC, "hipHostMalloc of the descriptor table failed");
    }
    std::memcpy(B->h_desc, desc.data(), sizeof(BatchDesc) * B->ninst);
    MWG_HIP(hipMemcpy(B->d_desc, desc.data(), sizeof(BatchDesc) * B->ninst, hipMemcpyHostToDevice));
    MWG_TRY(B->arena.alloc(&p, sizeof(GridItem) * std::max<size_t>(items.size(), 1)));
    B->d_items = (GridItem *)p;
    if (!items.empty())
        MWG_HIP(hipMemcpy(B->d_items, items.data(), sizeof(GridItem) * items.size(), hipMemcpyHostToDevice));
    MWG_TRY(B->arena.alloc(&p, sizeof(BatchItem) * std::max<size_t>(ditems.size(), 1)));
    B->d_ditems = (BatchItem *)p;
    if (!ditems.empty())
        MWG_HIP(hipMemcpy(B->d_ditems, ditems.data(), sizeof(BatchItem) * ditems.size(), hipMemcpyHostToDevice));
    {
        // (instance, block) pairs of flush-2 instances: all merge blocks, then all zero
        // blocks; (instance, tile) pairs of the zero tiles of flush-3 instances
        std::vector<int2> mp, zt;
        for (int i = 0; i < B->ninst; i++) {
            const Instance &I = *P.inst[i];
            if (I.L.flush == 3) {
                for (int32_t t : I.h_ozero) zt.push_back(make_int2(i, t));
                continue;
            }
            for (int k = 0; k < I.n_mblocks; k++) mp.push_back(make_int2(i, I.h_mblocks[k]));
        }
        B->merge_blocks = (int64_t)mp.size();
        for (int i = 0; i < B->ninst; i++)
            if (P.inst[i]->L.flush != 3)
                for (int k = P.inst[i]->n_mblocks; k < (int)P.inst[i]->h_mblocks.size(); k++)
                    mp.push_back(make_int2(i, P.inst[i]->h_mblocks[k]));
        B->zero_blocks = (int64_t)mp.size() - B->merge_blocks;
        B->ztiles = (int64_t)zt.size();
        MWG_TRY(B->arena.alloc(&p, sizeof(int2) * std::max<size_t>(mp.size(), 1)));
        B->d_mpairs = (int2 *)p;
        if (!mp.empty())
            MWG_HIP(hipMemcpy(B->d_mpairs, mp.data(), sizeof(int2) * mp.size(), hipMemcpyHostToDevice));
        MWG_TRY(B->arena.alloc(&p, sizeof(int2) * std::max<size_t>(zt.size(), 1)));
        B->d_ztiles = (int2 *)p;
        if (!zt.empty())
            MWG_HIP(hipMemcpy(B->d_ztiles, zt.data(), sizeof(int2) * zt.size(), hipMemcpyHostToDevice));
    }
    MWG_TRY(B->arena.alloc(&p, sizeof(int64_t) * pstart.size()));
    B->d_pro_start = (int64_t *)p;
    MWG_HIP(hipMemcpy(B->d_pro_start, pstart.data(), sizeof(int64_t) * pstart.size(), hipMemcpyHostToDevice));
    MWG_HIP(hipEventCreateWithFlags(&B->desc_ev, hipEventDisableTiming));
    MWG_HIP(hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking));
    MWG_HIP(hipStreamCreateWithFlags(&B->side, hipStreamNonBlocking));
    MWG_HIP(hipEventCreateWithFlags(&B->fork, hipEventDisableTiming));
    MWG_HIP(hipEventCreateWithFlags(&B->join, hipEventDisableTiming));
    // launch shapes
    B->grid_lds = 4 * ((size_t)B->O * 8 + (size_t)B->waves * B->per_wave);
    B->grid_blocks = std::max(1, (B->nitems + B->waves - 1) / B->waves);
    const int Rd = B->T + B->W - 1;
    if (B->npol == 4 && (B->W == 3 || B->W == 5 || B->W == 7)) {  // the run degridder
        const int nw = B->dthreads / 64;
        B->degrid_lds = degrid_runs_lds(B->npol, B->T, B->W, B->O, nw, 0);
        B->ant_in_lds = (max_nant > 0 && degrid_runs_lds(B->npol, B->T, B->W, B->O, nw, max_nant) <= 64 * 1024) ? 1 : 0;
        if (B->ant_in_lds) B->degrid_lds = degrid_runs_lds(B->npol, B->T, B->W, B->O, nw, max_nant);
    } else {
        B->degrid_lds = sizeof(float2) * (size_t)B->npol * Rd * Rd + 4 * (size_t)((B->O * B->W + 1) & ~1);
        B->ant_in_lds = (max_nant > 0 && B->degrid_lds + sizeof(float2) * (size_t)max_nant <= 64 * 1024) ? 1 : 0;
        if (B->ant_in_lds) B->degrid_lds += sizeof(float2) * (size_t)max_nant;
    }
    return Status::Ok();
}

Status batch_grid(Plan &P, const void *const *vis, const void *const *gains, void *const *grid, int accumulate,
                  hipStream_t s) {
    Batch &B = *(Batch *)P.batch;
    MWG_TRY(refresh_desc(B, vis, gains, nullptr, grid, nullptr, nullptr, accumulate, s));
    return run(B, false, 0, s);
}

Status batch_degrid(Plan &P, const void *const *grid, const void *const *gains, const void *const *vis_in,
                    void *const *vis_out, void *const *grad_gains, hipStream_t s) {
    Batch &B = *(Batch *)P.batch;
    // grid is read-only here; the descriptor's grid slot carries it
    MWG_TRY(refresh_desc(B, nullptr, gains, vis_in, (void *const *)grid, vis_out, grad_gains, 0, s));
    int64_t ndrop = 0;
    for (Instance *I : P.inst) ndrop += I->ngroups - I->nkept;
    return run(B, true, ndrop, s);
}

void batch_release(Plan &P) {
    Batch *B = (Batch *)P.batch;
    if (!B) return;
    if (B->desc_pending && B->desc_ev) (void)hipEventSynchronize(B->desc_ev);
    if (B->x_grid) (void)hipGraphExecDestroy(B->x_grid);
    if (B->x_degrid) (void)hipGraphExecDestroy(B->x_degrid);
    if (B->desc_ev) (void)hipEventDestroy(B->desc_ev);
    if (B->cap) (void)hipStreamDestroy(B->cap);
    if (B->side) (void)hipStreamDestroy(B->side);
    if (B->fork) (void)hipEventDestroy(B->fork);
    if (B->join) (void)hipEventDestroy(B->join);
    if (B->h_desc) (void)hipHostFree(B->h_desc);
    B->arena.release();
    delete B;
    P.batch = nullptr;
}

} // namespace mwg
