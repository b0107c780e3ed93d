// Launch autotuner: times candidate gridder launches on the plan's own positions (the
// visibility values do not change the work, so a buffer of ones stands in for them) and
// keeps the fastest. Tile size changes re-sort the plan; split, waves, schedule and flush
// changes only rebuild the work list. Results can be cached in a text file of one JSON
// object per line (path in MW_TUNE_CACHE).
#include "internal.h"
#include "tune_cache.h"

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

namespace mwg {

Status resolve_launch(const Instance &I, const mw_tuning *t, Launch *out);

namespace {

__global__ void k_fill_ones(float2 *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = make_float2(1.0f, 0.0f);
}

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

std::string cache_key(const Instance &I) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t prop;
    std::string arch = "gpu";
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
    const int mag = I.nkept > 0 ? (int)std::lround(std::log2((double)I.nkept)) : 0;
    char buf[256];
    snprintf(buf, sizeof buf, "%s/%dx%d/W%d/O%d/p%d/n2^%d", arch.c_str(), I.nx, I.ny, I.W, I.O, I.npol, mag);
    return buf;
}

bool cache_lookup(const char *path, const std::string &key, Launch *L) {
    TuneRecord r;
    if (!tune_cache_lookup(path, key.c_str(), &r)) return false;
    L->tile = r.tile;
    L->split = r.split;
    L->wg_waves = r.wg_waves;
    L->order = r.order;
    L->variant = r.variant;
    L->flush = r.flush;
    L->schedule = r.schedule;
    return true;
}

void cache_store(const char *path, const std::string &key, const Launch &c, float ms) {
    tune_cache_store(path, key.c_str(), TuneRecord{c.tile, c.split, c.wg_waves, c.order, c.variant, c.flush, c.schedule},
                     ms);
}

Status elapsed(hipEvent_t e0, hipEvent_t e1, float *ms) {
    MWG_HIP(hipEventSynchronize(e1));
    MWG_HIP(hipEventElapsedTime(ms, e0, e1));
    return Status::Ok();
}

// One warm-up launch, then the mean of three timed ones (HIP events on s).
template <class F>
Status time_calls(F &&call, hipStream_t s, float *ms) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    Status st;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        st = make_error(MW_ERR_HIP, "hipEventCreate failed");
    if (st.ok()) st = call();
    if (st.ok() && hipEventRecord(e0, s) != hipSuccess) st = make_error(MW_ERR_HIP, "hipEventRecord");
    for (int r = 0; r < 3 && st.ok(); r++) st = call();
    if (st.ok() && hipEventRecord(e1, s) != hipSuccess) st = make_error(MW_ERR_HIP, "hipEventRecord");
    float t = 0.f;
    if (st.ok()) st = elapsed(e0, e1, &t);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    *ms = t / 3.0f;
    return st;
}

// Candidate launches: the default launch (all fields zero) first, then the grid of tile
// sizes, waves per workgroup, work-item splits and schedules of the instance's kernel. The
// caller's non-zero fields stay fixed; flush stays 2 (the bit-reproducible merge) unless the
// caller set it to 1.
std::vector<mw_tuning> candidates(const Instance &I, const mw_tuning &user, bool batch) {
    std::vector<mw_tuning> out;
    auto push = [&](mw_tuning t) {
        if (user.tile) t.tile = user.tile;
        if (user.split) t.split = user.split;
        if (user.wg_waves) t.wg_waves = user.wg_waves;
        if (user.order) t.order = user.order;
        if (user.variant) t.variant = user.variant;
        if (user.schedule) t.schedule = user.schedule;
        t.flush = user.flush ? user.flush : (t.flush ? t.flush : 0);
        t.autotune = 0;
        for (const mw_tuning &o : out)
            if (std::memcmp(&o, &t, sizeof t) == 0) return;
        out.push_back(t);
    };
    push(mw_tuning{});
    const bool v4 = I.W >= 3 && I.W <= 7;
    const std::vector<int> tiles = v4 ? (batch ? std::vector<int>{8, 16, 32} : std::vector<int>{8, 16})
                                      : std::vector<int>{16, 32, 64};
    const std::vector<int> waves = batch ? std::vector<int>{4, 8} : std::vector<int>{4, 8, 16};
    const std::vector<int> splits = {0, 2048, 8192, 16384};
    for (int tile : tiles)
        for (int w : waves)
            for (int split : splits)
                for (int sched : {1, 2, 3}) {
                    if (!v4 && sched != 1) continue;
                    if (batch && sched != 1) continue;  // the batched kernel takes one item per wave
                    mw_tuning t{};
                    t.tile = tile;
                    t.wg_waves = w;
                    t.split = split;
                    t.schedule = sched;
                    t.order = 3;
                    t.variant = v4 ? 4 : (I.W * I.W <= 64 ? 1 : 3);
                    t.flush = 2;
                    push(t);
                }
    return out;
}

mw_tuning from_launch(const Launch &L) {
    mw_tuning t{};
    t.tile = L.tile;
    t.split = L.split;
    t.wg_waves = L.wg_waves;
    t.order = L.order;
    t.variant = L.variant;
    t.flush = L.flush;
    t.schedule = L.schedule;
    return t;
}

constexpr mw_tuning kDefault{};

} // namespace

bool batch_compatible(const Plan &P) {
    if (P.inst.size() < 2) return false;
    const Instance &I0 = *P.inst[0];
    for (const Instance *I : P.inst)
        if (I->stacks || I0.stacks || I->npol != I0.npol || I->W != I0.W || I->O != I0.O) return false;
    return I0.W >= 3 && I0.W <= 7;
}

Status autotune(Instance &I, const mw_tuning &user, hipStream_t s) {
    if (I.stacks || I.nkept == 0) return Status::Ok();
    const char *path = std::getenv("MW_TUNE_CACHE");
    const std::string key = cache_key(I);
    Launch cached;
    if (path && cache_lookup(path, key, &cached)) {
        const mw_tuning t = from_launch(cached);
        Launch L;
        if (resolve_launch(I, &t, &L).ok()) return rebuild_schedule(I, L, s);
    }
    DevBuf vis, grid;
    const int64_t nv = I.ngroups * I.npol;
    if (hipMalloc(&vis.p, sizeof(float2) * (size_t)std::max<int64_t>(nv, 1)) != hipSuccess ||
        hipMalloc(&grid.p, sizeof(float2) * (size_t)I.npol * I.nx * I.ny) != hipSuccess) {
        (void)hipGetLastError();
        return make_error(MW_ERR_ALLOC, "autotune buffers");
    }
    if (nv > 0) {
        hipLaunchKernelGGL(k_fill_ones, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, s, (float2 *)vis.p, nv);
        MWG_HIP(hipGetLastError());
    }
    float best_ms = 1e30f;
    Launch best = I.L;
    bool have = false;
    for (const mw_tuning &t : candidates(I, user, false)) {
        Launch L;
        if (!resolve_launch(I, &t, &L).ok()) continue;  // does not fit this instance
        MWG_TRY(rebuild_schedule(I, L, s));
        float ms = 0.f;
        MWG_TRY(time_calls([&] { return launch_grid(I, (const float2 *)vis.p, nullptr, (float2 *)grid.p, 0, s); },
                           s, &ms));
        if (!have || ms < best_ms) {
            best_ms = ms;
            best = L;
            have = true;
        }
    }
    MWG_TRY(rebuild_schedule(I, best, s));
    if (path && have) cache_store(path, key, best, best_ms);
    return Status::Ok();
}

// A plan of several instances that can share one launch is tuned as a whole: every
// candidate is applied to all instances and the batched sequence (one gridder launch over
// all instances' work items, then the merge) is timed. The plan ends batched, or the call
// fails; it never falls back to one launch sequence per instance behind the caller's back.
Status autotune_plan(Plan &P, const mw_tuning &user, hipStream_t s) {
    if (!batch_compatible(P)) {
        for (Instance *I : P.inst) MWG_TRY(autotune(*I, user, s));
        return P.inst.size() > 1 ? batch_prepare(P, s) : Status::Ok();
    }
    // the untuned batch (the default launch with the batch's own tile rule) is the baseline
    MWG_TRY(batch_prepare(P, s));
    int64_t kept = 0, cells = 0;
    for (const Instance *I : P.inst) {
        kept += I->nkept;
        cells += (int64_t)I->nx * I->ny;
    }
    char kb[256];
    {
        int dev = 0;
        (void)hipGetDevice(&dev);
        hipDeviceProp_t prop;
        std::string arch = "gpu";
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
        snprintf(kb, sizeof kb, "%s/batch%zu/W%d/O%d/p%d/n2^%d/c2^%d", arch.c_str(), P.inst.size(), P.inst[0]->W,
                 P.inst[0]->O, P.inst[0]->npol, kept > 0 ? (int)std::lround(std::log2((double)kept)) : 0,
                 (int)std::lround(std::log2((double)std::max<int64_t>(cells, 1))));
    }
    const std::string key = kb;
    const char *path = std::getenv("MW_TUNE_CACHE");
    auto apply = [&](const mw_tuning &t) -> Status {
        std::vector<Launch> Ls(P.inst.size());
        for (size_t i = 0; i < P.inst.size(); i++) {
            Status r = resolve_launch(*P.inst[i], &t, &Ls[i]);
            if (!r.ok()) return r;
        }
        batch_release(P);
        for (size_t i = 0; i < P.inst.size(); i++) {
            MWG_TRY(rebuild_schedule(*P.inst[i], Ls[i], s));
            P.inst[i]->tile_fixed = true;  // keep the candidate's tile in the batch
        }
        return batch_prepare(P, s);
    };
    if (!P.batch) return make_error(MW_ERR_STATE, "the plan's instances did not form a batch");
    Launch cached;
    if (path && cache_lookup(path, key, &cached)) {
        const mw_tuning t = from_launch(cached);
        if (std::memcmp(&t, &kDefault, sizeof t) == 0) return Status::Ok();  // the untuned batch won
        if (apply(t).ok() && P.batch) return Status::Ok();
        batch_release(P);
        MWG_TRY(batch_prepare(P, s));  // a stale entry: search again
        if (!P.batch) return make_error(MW_ERR_STATE, "the plan's instances did not form a batch");
    }
    std::vector<DevBuf> vis(P.inst.size()), grid(P.inst.size());
    std::vector<const void *> vp(P.inst.size());
    std::vector<void *> gp(P.inst.size());
    for (size_t i = 0; i < P.inst.size(); i++) {
        const Instance &I = *P.inst[i];
        const int64_t nv = I.ngroups * I.npol;
        if (hipMalloc(&vis[i].p, sizeof(float2) * (size_t)std::max<int64_t>(nv, 1)) != hipSuccess ||
            hipMalloc(&grid[i].p, sizeof(float2) * (size_t)I.npol * I.nx * I.ny) != hipSuccess) {
            (void)hipGetLastError();
            return make_error(MW_ERR_ALLOC, "autotune buffers");
        }
        if (nv > 0) {
            hipLaunchKernelGGL(k_fill_ones, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, s,
                               (float2 *)vis[i].p, nv);
            MWG_HIP(hipGetLastError());
        }
        vp[i] = vis[i].p;
        gp[i] = grid[i].p;
    }
    auto run = [&] { return batch_grid(P, vp.data(), nullptr, gp.data(), 0, s); };
    float best_ms = 0.f;
    MWG_TRY(time_calls(run, s, &best_ms));
    mw_tuning best = kDefault;
    bool best_is_default = true;
    std::vector<Launch> base(P.inst.size());
    for (size_t i = 0; i < P.inst.size(); i++) base[i] = P.inst[i]->L;
    for (const mw_tuning &t : candidates(*P.inst[0], user, true)) {
        if (std::memcmp(&t, &kDefault, sizeof t) == 0) continue;  // the baseline, timed above
        if (!apply(t).ok() || !P.batch) continue;  // does not fit some instance
        float ms = 0.f;
        MWG_TRY(time_calls(run, s, &ms));
        if (ms < best_ms) {
            best_ms = ms;
            best = t;
            best_is_default = false;
        }
    }
    if (best_is_default) {
        batch_release(P);
        for (size_t i = 0; i < P.inst.size(); i++) MWG_TRY(rebuild_schedule(*P.inst[i], base[i], s));
        MWG_TRY(batch_prepare(P, s));
    } else {
        MWG_TRY(apply(best));
    }
    if (!P.batch) return make_error(MW_ERR_STATE, "the tuned launch did not form a batch");
    if (path) {
        // the candidate itself (split 0 = each instance's own default), not instance 0's
        // resolved launch
        Launch c;
        c.tile = best.tile;
        c.split = best.split;
        c.wg_waves = best.wg_waves;
        c.order = best.order;
        c.variant = best.variant;
        c.flush = best.flush;
        c.schedule = best.schedule;
        cache_store(path, key, c, best_ms);
    }
    return Status::Ok();
}

} // namespace mwg
