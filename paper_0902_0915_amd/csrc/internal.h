// Internal declarations of libmwagrid (not installed; the public ABI is include/mwagrid.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "mwagrid.h"

namespace mwg {

// ------------------------------------------------------------------------------------------
// Errors: every internal step returns a Status; the ABI layer turns it into mw_status and
// records the message for mw_last_error().
// ------------------------------------------------------------------------------------------
struct Status {
    mw_status code = MW_OK;
    std::string msg;
    bool ok() const { return code == MW_OK; }
    static Status Ok() { return {}; }
};
Status make_error(mw_status code, const char *fmt, ...);

#define MWG_HIP(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return ::mwg::make_error(MW_ERR_HIP, "%s failed: %s (%s:%d)", #expr,             \
                                     hipGetErrorString(e_), __FILE__, __LINE__);              \
    } while (0)

#define MWG_TRY(expr)                                                                         \
    do {                                                                                      \
        ::mwg::Status s_ = (expr);                                                            \
        if (!s_.ok()) return s_;                                                              \
    } while (0)

// Device allocation tracked per instance so that plan_bytes can be reported.
struct DevArena {
    std::vector<void *> ptrs;
    int64_t bytes = 0;
    char *chunk = nullptr;  // the current chunk of small arrays and what is left of it
    size_t chunk_left = 0;
    Status alloc(void **p, size_t nbytes);
    void release();
};

// Temporary device memory of plan construction (sort keys, scan workspaces, counters).
// Inside a TmpScope, temporaries on the scope's stream are carved last-in first-out from
// blocks that the scope owns and frees when it ends, so a plan of many small instances does
// not pay a hipMalloc/hipFree pair per temporary. Memory a temporary gives back may be handed
// out again while kernels that read it are still queued: the next user is queued behind them
// on the same stream. Outside a scope, or on another stream, a temporary is its own hipMalloc
// and its destructor waits for the device (hipFree does).
struct TmpPool;
struct DevTmp {
    void *p = nullptr;
    DevTmp() = default;
    DevTmp(const DevTmp &) = delete;
    DevTmp &operator=(const DevTmp &) = delete;
    ~DevTmp() { release(); }
    Status alloc(size_t nbytes, hipStream_t s);
    void release();
    bool pooled() const { return pool != nullptr; }
    template <class T> T *as() const { return (T *)p; }

  private:
    TmpPool *pool = nullptr;
};

class TmpScope {
  public:
    // first_block: size of the pool's first block (0: the default); a build that knows its
    // peak need gets it in one allocation (each hipMalloc/hipFree pair costs ~0.3 ms)
    explicit TmpScope(hipStream_t s, size_t first_block = 0);
    ~TmpScope();
    TmpScope(const TmpScope &) = delete;
    TmpScope &operator=(const TmpScope &) = delete;

  private:
    TmpPool *own = nullptr;  // null when an enclosing scope is already active on this thread
};

// Runs job(i, stream) for every i in [0, n) on up to 8 host threads, each issuing to a stream
// of its own that first waits for the work already on `after`, each with its own pool of
// temporaries (workers.cpp). Jobs must touch disjoint state. Returns the first error; all
// device work of the jobs has finished when it returns.
Status parallel_instances(int device, int n, hipStream_t after, const std::function<Status(int, hipStream_t)> &job,
                          size_t tmp_first_block = 0);
// A first temporary block that holds one instance's build: its sort (16 bytes per group and
// a little more) and the per-cell tables of its grid.
size_t plan_tmp_hint(int64_t ngroups, int nx, int ny);

// Smallest r with 2^r >= v (the exponent of a power-of-two tile size).
inline int ilog2(int v) {
    int r = 0;
    while ((1 << r) < v) r++;
    return r;
}

// Merge pass: blocks of kMergeB x kMergeB cells; a block meets at most kMergeTiles tiles
// (5 x 5 for tiles of 8 or more cells and supports up to 15).
constexpr int kMergeB = 16;
constexpr int kMergeTiles = 25;

// Packed per-group position: cx | cy << 12 | (px + O/2) << 24 | (py + O/2) << 28.
constexpr uint32_t kDropped = 0xFFFFFFFFu;
__host__ __device__ inline uint32_t pack_pos(int cx, int cy, int pxo, int pyo) {
    return (uint32_t)cx | ((uint32_t)cy << 12) | ((uint32_t)pxo << 24) | ((uint32_t)pyo << 28);
}

// Launch configuration of the gridder / degridder for one instance.
struct Launch {
    int tile = 32;     // T (power of two)
    int split = 8192;  // max groups per work item
    int wg_waves = 8;  // waves per workgroup
    int order = 1;     // 1 cell-sorted, 2 input order within tile, 3 cell-sorted along the radius
    int variant = 1;   // gridder variant
    int flush = 1;     // 1 atomic, 2 deterministic merge, 3 owner tiles (written once, no merge)
    int schedule = 1;  // 1 largest first, 2 Z-order chunks per XCD, 3 workgroup-cooperative items
};

struct WorkItem {
    int32_t tile, begin, end, pad;
};

struct Instance {
    // description (copied from mw_instance)
    int nx = 0, ny = 0, npol = 1, nchan = 1, W = 0, O = 1, h = 0, nant = 0;
    int64_t nrow = 0, ngroups = 0;
    double du = 0, dv = 0;
    bool stacks = false, has_weights = false, has_ants = false;
    int nkernel = 0, max_support = 0;
    // counts
    int64_t nkept = 0, nflagged = 0, noutside = 0;
    // launch
    Launch L;
    bool tile_fixed = false;  // the caller chose the tile (or asked the autotuner)
    bool flush_fixed = false; // the caller chose the flush
    int ntx = 0, nty = 0, ntiles_nonempty = 0, nwork = 0;
    int64_t ntiles8 = 0;     // occupied 8 x 8 tiles (counted for plans of several instances)
    bool scheduled = false;  // sort and work list built for the launch L
    int max_work_groups = 0;  // largest work item
    int sorted_tile = 0, sorted_order = 0;   // the (tile, order) perm is currently sorted by
    std::vector<int32_t> h_tstart, h_tend;  // tile bounds of that sort (host)
    size_t cap_work = 0, cap_tiles = 0;      // capacities of work / tile_work / work_ids
    // optional timing of the gridder and merge launches (mw_plan_set_timing)
    bool timing = false;
    hipEvent_t tev[3] = {nullptr, nullptr, nullptr};
    bool timed = false;
    int xcd_start[9] = {0};   // schedule 2: first logical workgroup of each XCD's chunk
    int xcd_wgs = 0;          // schedule 2: workgroups per XCD in the launch grid
    int coop_wgs = 0;         // schedule 3: workgroups in the launch grid
    size_t cap_coop = 0;      // schedule 3: capacity of coop (wave slots)
    // device arrays (owned by arena)
    DevArena arena;
    uint32_t *pos = nullptr;      // [ngroups] packed, original order
    uint32_t *perm = nullptr;     // [nkept] sorted -> original group
    uint32_t *spos = nullptr;     // [nkept] packed, sorted
    float *sw = nullptr;          // [nkept] weights, sorted (or null)
    uint32_t *sant = nullptr;     // [nkept] ant1 | ant2 << 16, sorted (or null)
    uint32_t *skid = nullptr;     // [nkept] kernel id, sorted (stacks)
    uint32_t *dropped = nullptr;  // [ngroups - nkept] original indices of dropped groups
    uint32_t *scode = nullptr;    // [nkept + 64] per sorted group: LDS cell offset | px*W << 16 | py*W << 24
    float *w_orig = nullptr;      // [ngroups] weights in input order (or null)
    uint32_t *ant_orig = nullptr; // [nrow] ant1 | ant2 << 16 (or null)
    int32_t *kidx_orig = nullptr; // [ngroups] kernel index (stacks)
    WorkItem *work = nullptr;     // [nwork]
    int2 *coop = nullptr;         // schedule 3: [coop_wgs * wg_waves] per wave slot: (item or -1,
                                  //   k | nsub << 8), wave k of the nsub consecutive waves of item
    int32_t *tile_work = nullptr; // [ntiles + 1] CSR: work items of each tile (merge flush)
    int32_t *work_ids = nullptr;  // [nwork] work item ids grouped by tile
    int32_t *mblocks = nullptr;   // merge blocks (by * bpr + bx): those some work item reaches,
    int n_mblocks = 0;            //   then the n_zblocks that none reaches (written as zeros)
    int n_zblocks = 0;
    // flush 3 (owner tiles): per output tile, the sorted groups whose footprint reaches it
    int owner_tile = 0;           // tile size the owner lists were built for (0: none)
    int nowork = 0;               // owner work items: output tiles with candidates
    int n_ozero = 0;              // output tiles without candidates (written as zeros)
    int max_owner_groups = 0;     // largest owner work item
    int64_t npairs_owner = 0;
    WorkItem *owork = nullptr;    // [nowork] {tile, begin, end} into the pair arrays, largest first
    uint32_t *pperm = nullptr;    // [npairs] original group of each (output tile, group) pair
    uint32_t *pcode = nullptr;    // [npairs] its code relative to the output tile's LDS tile
    float *psw = nullptr;         // [npairs] weights (or null)
    uint32_t *psant = nullptr;    // [npairs] antenna pairs (or null)
    int32_t *ozero = nullptr;     // [n_ozero] output tiles without candidates
    size_t cap_pairs = 0, cap_owork = 0, cap_ozero = 0;
    // host copies of the lists built on the host (the batched plan reads them back from here)
    std::vector<WorkItem> h_work, h_owork;
    std::vector<int32_t> h_mblocks, h_ozero, h_tw, h_ids;
    std::vector<int2> h_coop;
    std::vector<float> h_taps2d, h_tabpad, h_tab8;  // sources of the table uploads
    float *partial = nullptr;     // merge flush scratch: [nwork][R*R][2*npol] (cell-major)
    size_t partial_bytes = 0;
    float *taps2d = nullptr;      // [O*O][64] separable taps products (W <= 7 lanes layout)
    float *tab = nullptr;         // [O][W] + 8 floats of padding
    float *tab8 = nullptr;        // [O][8]: rows padded to 8 floats (W <= 7), 32-byte aligned
    float *corrx = nullptr, *corry = nullptr;
    float2 *kstack = nullptr;     // stacks: complex taps
    uint32_t *pairs = nullptr;    // stacks: candidate group of each (tile, group) pair, by tile
    int64_t npairs = 0;
    int64_t *koff = nullptr;
    int32_t *ksup = nullptr;
    // w-stacking: the instance grids only groups with wlo <= w < whi (wavelengths)
    bool wsel = false;
    double wlo = 0, whi = 0;
    // prediction and calibration (calib.hip)
    double *uvw_d = nullptr;      // [nrow][3] metres
    double *kf_d = nullptr;       // [nchan] f / c, turns per metre
    // variant 6: the sorted arrays with every (cell, py) run of a work item padded to a
    // multiple of 4 entries (runs.hip); same work items, padded ranges
    int block_tile = 0;           // tile the padded schedule was built for (0: none)
    int64_t nblocked = 0, cap_blocked = 0;  // padded entries and their capacity
    size_t cap_bwork = 0;         // capacity of bwork
    WorkItem *bwork = nullptr;    // [nwork]
    uint32_t *bperm = nullptr;    // [nblocked + 64] group, or 0xFFFFFFFF for a padding entry
    uint32_t *bcode = nullptr;    // [nblocked + 64] codes as scode (a padding entry: its run's)
    float *bsw = nullptr;         // [nblocked] weights (or null)
    uint32_t *bsant = nullptr;    // [nblocked] antenna pairs (or null)
    int64_t cal_npair = 0;        // antenna pairs (baselines) among the rows
    uint32_t *cal_pant = nullptr; // [npair] a1 | a2 << 16
    int32_t *cal_pstart = nullptr; // [npair + 1] CSR of each pair's rows
    int32_t *cal_prows = nullptr; // [nrow]
    int32_t *cal_start = nullptr; // [nant + 1] CSR of each antenna's pairs
    int32_t *cal_entry = nullptr; // [2 npair] pair << 1 | (0: the pair's ant1, 1: its ant2)
    int32_t *cal_partner = nullptr; // [2 npair] the pair's other antenna
    float4 *cal_pq = nullptr;     // [npair] per-pair sums (Re P, Im P, Q, 0)
    float2 *cal_g = nullptr;      // [nant] second gain buffer of the iteration
    double *cal_red = nullptr;    // [2 nant] per-antenna |step|^2 and |g|^2 of the last iteration
    void *src_d = nullptr, *src_h = nullptr;  // source table, device and pinned host staging
    size_t src_cap = 0;
    hipEvent_t src_ev = nullptr;  // guards src_h until its upload has read it
    bool src_pending = false;
    // host copies for export
    std::vector<float> h_tab, h_corrx, h_corry;
    // image plans (rocFFT); opaque here
    void *fft = nullptr;                          // rocFFT plans (grids of other sizes)
    float2 *twx = nullptr, *twy = nullptr;        // two-pass transform twiddles (power-of-two grids)
};

struct Plan {
    int device = 0;
    std::vector<Instance *> inst;
    // batched form (ninst > 1)
    void *batch = nullptr;
};

// pswf.cpp
void prolate_tables(int W, int O, int nx, int ny, std::vector<float> &table,
                    std::vector<float> &corr_x, std::vector<float> &corr_y);

// plan.hip
// schedule: build the sort and work list now (false: the caller does, with schedule_instance,
// once the launch is settled); count_tiles: count the occupied 8 x 8 tiles (ntiles8)
Status build_instance(Instance &I, const mw_instance &d, const mw_tuning *t, hipStream_t s, bool schedule = true,
                      bool count_tiles = false);
Status schedule_instance(Instance &I, const Launch &L, hipStream_t s);
// runs.hip: the block-padded work list of variant 6 from the current sort and codes
Status build_block_schedule(Instance &I, hipStream_t s);
Status rebuild_schedule(Instance &I, const Launch &L, hipStream_t s);

// stack.hip
Status build_stack_schedule(Instance &I, const Launch &L, hipStream_t s);
Status launch_grid_stack(Instance &I, const float2 *vis, const float2 *gains, float2 *grid,
                         int accumulate, hipStream_t s);
Status launch_degrid_stack(Instance &I, const float2 *grid, const float2 *gains,
                           const float2 *vis_in, float2 *vis_out, float2 *grad_gains,
                           hipStream_t s);
size_t stack_lds(int npol, int T, int waves);

// grid.hip
Status launch_grid(Instance &I, const float2 *vis, const float2 *gains, float2 *grid,
                   int accumulate, hipStream_t s);
// The same launch with the merge flush's partial tiles in caller-given device memory of
// partial_cap bytes (no allocation; MW_ERR_UNSUPPORTED if the plan needs more).
Status launch_grid_into(Instance &I, const float2 *vis, const float2 *gains, float2 *grid, int accumulate,
                        float *partial, size_t partial_cap, hipStream_t s);
// Device address of the library's static scratch array on the current device (looked up once
// per device) and its size in bytes.
Status static_scratch(void **ptr, size_t *bytes);
Status launch_fill_zero(void *ptr, size_t nbytes, hipStream_t s);

// degrid.hip
Status launch_degrid(Instance &I, const float2 *grid, const float2 *gains, const float2 *vis_in,
                     float2 *vis_out, float2 *grad_gains, hipStream_t s);

// image.cpp / image.hip
Status image_prepare(Instance &I);
Status launch_image(Instance &I, const float2 *in, float2 *out, int direction, int correct,
                    hipStream_t s);
void image_release(Instance &I);
bool fft2d_supported(int nx, int ny);
Status fft2d_twiddles(DevArena &arena, int n, float2 **out, hipStream_t s);
Status launch_fft2d(const float2 *in, float2 *out, int nx, int ny, int npol, const float2 *twx,
                    const float2 *twy, const float *corrx, const float *corry, int direction, int correct,
                    hipStream_t st);
Status launch_image_scale(const float2 *in, float2 *out, int nx, int ny, int npol,
                          const float *corrx, const float *corry, int checker, int divide,
                          hipStream_t s);

// calib.hip
Status build_calibration(Instance &I, const double *uvw_dev, const double *freq_dev, const int32_t *a1_dev,
                         const int32_t *a2_dev, hipStream_t s);
Status launch_predict(Instance &I, const double *sources, int nsrc, const float2 *gains, float2 *out,
                      int accumulate, hipStream_t s);
Status launch_solve_gains(Instance &I, const float2 *vis, const float2 *model, const float *weights, float2 *gains,
                          int niter, float *rel, hipStream_t s);
Status launch_peel(Instance &I, const float2 *vis, const double *sources_host, int nsrc, const float *weights,
                   int niter, float2 *resid, float2 *gains, float *rel, hipStream_t s);

// wstack.hip
Status launch_wstack_combine(Plan &P, const void *const *images, float2 *out, int accumulate, hipStream_t s);

// weighting.hip
Status apply_density_weighting(Instance &I, int mode, float robust, const float *w_in, float *w_out, hipStream_t s);

// owner.hip
Status build_owner_schedule(Instance &I, int64_t cap, bool *built, hipStream_t s);
Status launch_zero_tiles(const Instance &I, float2 *grid, hipStream_t s);

// stokes.hip
Status launch_stokes(const Instance &I, const float2 *images, const float2 *jones, float *out, hipStream_t s);

// batched.cpp
Status batch_prepare(Plan &P, hipStream_t s);
Status batch_grid(Plan &P, const void *const *vis, const void *const *gains, void *const *grid,
                  int accumulate, hipStream_t s);
Status batch_degrid(Plan &P, const void *const *grid, const void *const *gains,
                    const void *const *vis_in, void *const *vis_out, void *const *grad_gains,
                    hipStream_t s);
void batch_release(Plan &P);

// tuner.cpp
Status autotune(Instance &I, const mw_tuning &user, hipStream_t s);
Status autotune_plan(Plan &P, const mw_tuning &user, hipStream_t s);
bool batch_compatible(const Plan &P);

} // namespace mwg
