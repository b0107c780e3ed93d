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
Status launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);
Status ensure_partial(Instance &I, hipStream_t s);

namespace {

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
};

struct BatchItem {
    int32_t inst, item;
};

struct Batch {
    int ninst = 0, npol = 1, W = 7, O = 8, T = 8, waves = 8, STR = 0, PL = 0, nitems = 0;
    int dthreads = 256;  // threads per degridder workgroup
    int grid_blocks = 0;     // gridder workgroups (waves of them, one work item per wave)
    int64_t merge_blocks = 0, zero_blocks = 0, prologue_n = 0;
    int ant_in_lds = 0;
    size_t grid_lds = 0, degrid_lds = 0;
    DevArena arena;
    BatchDesc *d_desc = nullptr, *h_desc = nullptr; // h_desc: pinned host memory
    hipEvent_t desc_ev = nullptr;
    bool desc_pending = false;
    BatchItem *d_items = nullptr;
    int64_t *d_pro_start = nullptr;
    int2 *d_mpairs = nullptr; // (instance, block) of every merge block, then of every zero block
    const float *tab8 = nullptr;
    float tapk[16 * 8] = {0};
    hipStream_t cap = nullptr;
    hipGraphExec_t x_grid = nullptr, x_degrid = nullptr;
    bool use_graph = true;
};

struct BatchGridArgs {
    const BatchDesc *desc;
    const BatchItem *items;
    const float *tab8;
    int nitems, O, T, STR, PL;
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
    for (int i = tid; i < ntab; i += blockDim.x) ltab[i] = a.tab8[i];
    __syncthreads();
    const int w = blockIdx.x * (int)(blockDim.x >> 6) + wave;
    if (w >= a.nitems) return;
    const int R = a.T + W - 1;
    float *stage = smem + ntab + wave * wavetile_per_wave(NC, a.PL);
    const BatchItem it = a.items[w];
    const int inst = uni(it.inst), item = uni(it.item);
    const BatchDesc &d = a.desc[inst];
    const WorkItem wk = d.work[item];
    const int ntx = uni(d.ntx), wtile = uni(wk.tile);
    float *tile = stage + kStageFloats;
    for (int i = lane; i < NC * a.PL; i += 64) tile[i] = 0.0f;
    ItemCtx c;
    c.tile = tile;
    c.sv = stage;
    c.vis = uni(d.vis);
    c.gains = uni(d.gains);
    c.perm = uni(d.perm);
    c.scode = uni(d.scode);
    c.sant = uni(d.sant);
    c.sw = uni(d.sw);
    c.tapk = a.tapk;
    c.ltab = ltab;
    c.grid = uni(d.grid);
    c.partial = uni(d.partial) + (int64_t)item * NC * R * R;
    c.wb = uni(wk.begin);
    c.we = uni(wk.end);
    c.tx0 = (wtile % ntx) * a.T;
    c.ty0 = (wtile / ntx) * a.T;
    c.T = a.T;
    c.STR = a.STR;
    c.PL = a.PL;
    c.nx = uni(d.nx);
    c.ny = uni(d.ny);
    c.flush = 2;
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

template <int NPOL>
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
    degrid_item<NPOL>(a, d.work[it.item], smem);
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
    std::memcpy(a.tapk, B.tapk, sizeof a.tapk);
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
    if (B.zero_blocks > 0) {
        hipLaunchKernelGGL(k_zero_batched<NPOL>, dim3((unsigned)B.zero_blocks), dim3(kMergeB * kMergeB), 0, s,
                           B.d_desc, (const int2 *)B.d_mpairs + B.merge_blocks);
        MWG_HIP(hipGetLastError());
    }
    return Status::Ok();
}

template <int NPOL>
Status enqueue_degrid(Batch &B, int64_t ndrop_total, hipStream_t s) {
    if (B.prologue_n > 0) {
        hipLaunchKernelGGL(k_degrid_prologue<NPOL>, dim3((unsigned)((B.prologue_n + 255) / 256)), dim3(256), 0,
                           s, B.d_desc, (const int64_t *)B.d_pro_start, B.ninst, ndrop_total);
        MWG_HIP(hipGetLastError());
    }
    if (B.nitems > 0) {
        hipLaunchKernelGGL(k_degrid_batched<NPOL>, dim3(B.nitems), dim3(B.dthreads), B.degrid_lds, s, B.d_desc,
                           B.d_items, B.T, B.W, B.O, B.ant_in_lds);
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
    if (P.inst.size() < 2) return Status::Ok();
    // Sparse batches (fewer than 64 kept groups per non-empty 8 x 8 tile on average) take
    // 16 x 16 tiles: a quarter of the work items, each staging and flushing less halo per
    // group. The batch as a whole still has items enough to fill the chip, which one sparse
    // instance on its own does not, so single-instance plans keep 8 x 8.
    {
        bool retile = true;
        int64_t kept = 0, tiles = 0;
        for (const Instance *I : P.inst) {
            retile = retile && !I->stacks && !I->tile_fixed && I->L.variant == 4 && I->L.flush == 2 &&
                     I->L.tile == 8 && I->L.schedule == 1 &&
                     wavetiles_lds(I->npol, 16, I->W, I->O, I->L.wg_waves) <= 160 * 1024;
            kept += I->nkept;
            tiles += I->ntiles_nonempty;
        }
        if (retile && tiles > 0 && kept < 64 * tiles) {
            for (Instance *I : P.inst) {
                Launch L = I->L;
                L.tile = 16;
                MWG_TRY(rebuild_schedule(*I, L, s));
            }
        }
    }
    const Instance &I0 = *P.inst[0];
    for (const Instance *I : P.inst) {
        if (I->stacks || I->npol != I0.npol || I->W != I0.W || I->O != I0.O || I->L.variant != 4 ||
            I->L.flush != 2 || I->L.tile != I0.L.tile || I->L.wg_waves != I0.L.wg_waves)
            return Status::Ok();
    }
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
    B->tab8 = I0.tab8;
    for (int r = 0; r < I0.O; r++)
        for (int t = 0; t < I0.W; t++) B->tapk[r * 8 + t] = I0.h_tab[(size_t)r * I0.W + t];
    const char *ng = std::getenv("MW_NO_GRAPH");
    B->use_graph = !(ng && ng[0] == '1');
    // descriptors (fixed part)
    std::vector<BatchDesc> desc(B->ninst);
    std::vector<BatchItem> items;
    std::vector<int64_t> mstart(B->ninst + 1, 0), zstart(B->ninst + 1, 0), pstart(2 * B->ninst + 1, 0);
    int max_nant = 0;
    for (int i = 0; i < B->ninst; i++) {
        Instance &I = *P.inst[i];
        MWG_TRY(ensure_partial(I, s));
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
        max_nant = std::max(max_nant, I.nant);
        for (int w = 0; w < I.nwork; w++) items.push_back({i, w});
        mstart[i + 1] = mstart[i] + I.n_mblocks;
        zstart[i + 1] = zstart[i] + I.n_zblocks;
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
    {
        int64_t kept = 0;
        for (Instance *I : P.inst) kept += I->nkept;
        B->dthreads = degrid_threads(kept, B->nitems);
    }
    B->merge_blocks = mstart[B->ninst];
    B->zero_blocks = zstart[B->ninst];
    void *p;
    MWG_TRY(B->arena.alloc(&p, sizeof(BatchDesc) * B->ninst));
    B->d_desc = (BatchDesc *)p;
    if (hipHostMalloc((void **)&B->h_desc, sizeof(BatchDesc) * B->ninst, hipHostMallocDefault) != hipSuccess) {
        B->h_desc = nullptr;
        return make_error(MW_ERR_ALLOC, "hipHostMalloc of the descriptor table failed");
    }
    std::memcpy(B->h_desc, desc.data(), sizeof(BatchDesc) * B->ninst);
    MWG_HIP(hipMemcpy(B->d_desc, desc.data(), sizeof(BatchDesc) * B->ninst, hipMemcpyHostToDevice));
    MWG_TRY(B->arena.alloc(&p, sizeof(BatchItem) * std::max<size_t>(items.size(), 1)));
    B->d_items = (BatchItem *)p;
    if (!items.empty())
        MWG_HIP(hipMemcpy(B->d_items, items.data(), sizeof(BatchItem) * items.size(), hipMemcpyHostToDevice));
    {
        // (instance, block) pairs: all merge blocks, then all zero blocks
        std::vector<int2> mp;
        mp.reserve((size_t)(B->merge_blocks + B->zero_blocks));
        std::vector<std::vector<int32_t>> lists(B->ninst);
        for (int i = 0; i < B->ninst; i++) {
            const Instance &I = *P.inst[i];
            lists[i].resize((size_t)(I.n_mblocks + I.n_zblocks));
            if (!lists[i].empty())
                MWG_HIP(hipMemcpy(lists[i].data(), I.mblocks, 4 * lists[i].size(), hipMemcpyDeviceToHost));
            for (int k = 0; k < I.n_mblocks; k++) mp.push_back(make_int2(i, lists[i][k]));
        }
        for (int i = 0; i < B->ninst; i++)
            for (int k = P.inst[i]->n_mblocks; k < (int)lists[i].size(); k++) mp.push_back(make_int2(i, lists[i][k]));
        MWG_TRY(B->arena.alloc(&p, sizeof(int2) * std::max<size_t>(mp.size(), 1)));
        B->d_mpairs = (int2 *)p;
        if (!mp.empty())
            MWG_HIP(hipMemcpy(B->d_mpairs, mp.data(), sizeof(int2) * mp.size(), hipMemcpyHostToDevice));
    }
    MWG_TRY(B->arena.alloc(&p, sizeof(int64_t) * pstart.size()));
    B->d_pro_start = (int64_t *)p;
    MWG_HIP(hipMemcpy(B->d_pro_start, pstart.data(), sizeof(int64_t) * pstart.size(), hipMemcpyHostToDevice));
    MWG_HIP(hipEventCreateWithFlags(&B->desc_ev, hipEventDisableTiming));
    MWG_HIP(hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking));
    // launch shapes
    B->grid_lds = wavetiles_lds(B->npol, B->T, B->W, B->O, B->waves);
    B->grid_blocks = std::max(1, (B->nitems + B->waves - 1) / B->waves);
    const int Rd = B->T + B->W - 1;
    B->degrid_lds = sizeof(float2) * (size_t)B->npol * Rd * Rd + 4 * (size_t)((B->O * B->W + 1) & ~1);
    B->ant_in_lds = (max_nant > 0 && B->degrid_lds + sizeof(float2) * (size_t)max_nant <= 64 * 1024) ? 1 : 0;
    if (B->ant_in_lds) B->degrid_lds += sizeof(float2) * (size_t)max_nant;
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
    if (B->h_desc) (void)hipHostFree(B->h_desc);
    B->arena.release();
    delete B;
    P.batch = nullptr;
}

} // namespace mwg
