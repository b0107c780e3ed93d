// Launch autotuner: times candidate gridder launches on the plan's own positions (the
// visibility values do not change the work, so a buffer of ones stands in for them) and
// keeps the fastest. Tile size changes re-sort the plan; split, waves, schedule and flush
// changes only rebuild the work list. Results can be cached in a text file of one JSON
// object per line (path in MW_TUNE_CACHE).
#include "internal.h"

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
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
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        char k[256];
        Launch c;
        if (std::sscanf(line,
                        "{\"key\": \"%255[^\"]\", \"tile\": %d, \"split\": %d, \"wg_waves\": %d, "
                        "\"order\": %d, \"variant\": %d, \"flush\": %d, \"schedule\": %d}",
                        k, &c.tile, &c.split, &c.wg_waves, &c.order, &c.variant, &c.flush, &c.schedule) == 8 &&
            key == k) {
            *L = c; // the last matching line wins
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void cache_store(const char *path, const std::string &key, const Launch &c, float ms) {
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f,
                 "{\"key\": \"%s\", \"tile\": %d, \"split\": %d, \"wg_waves\": %d, \"order\": %d, "
                 "\"variant\": %d, \"flush\": %d, \"schedule\": %d, \"ms\": %.4f}\n",
                 key.c_str(), c.tile, c.split, c.wg_waves, c.order, c.variant, c.flush, c.schedule, ms);
    std::fclose(f);
}

Status time_launch(Instance &I, const float2 *vis, float2 *grid, hipStream_t s, float *ms) {
    hipEvent_t e0, e1;
    MWG_HIP(hipEventCreate(&e0));
    MWG_HIP(hipEventCreate(&e1));
    Status st = launch_grid(I, vis, nullptr, grid, 0, s); // warm-up
    if (st.ok() && hipEventRecord(e0, s) != hipSuccess) st = make_error(MW_ERR_HIP, "hipEventRecord");
    for (int r = 0; r < 3 && st.ok(); r++) st = launch_grid(I, vis, nullptr, grid, 0, s);
    if (st.ok() && hipEventRecord(e1, s) != hipSuccess) st = make_error(MW_ERR_HIP, "hipEventRecord");
    if (st.ok() && hipEventSynchronize(e1) != hipSuccess) st = make_error(MW_ERR_HIP, "hipEventSynchronize");
    float t = 0.f;
    if (st.ok() && hipEventElapsedTime(&t, e0, e1) != hipSuccess) st = make_error(MW_ERR_HIP, "hipEventElapsedTime");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = t / 3.0f;
    return st;
}

} // namespace

Status autotune(Instance &I, hipStream_t s) {
    if (I.stacks || I.nkept == 0) return Status::Ok();
    const char *path = std::getenv("MW_TUNE_CACHE");
    const std::string key = cache_key(I);
    Launch cached;
    if (path && cache_lookup(path, key, &cached)) {
        mw_tuning t{};
        t.tile = cached.tile;
        t.split = cached.split;
        t.wg_waves = cached.wg_waves;
        t.order = cached.order;
        t.variant = cached.variant;
        t.flush = cached.flush;
        t.schedule = cached.schedule;
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
    std::vector<mw_tuning> cands;
    const bool v4 = I.W >= 3 && I.W <= 7;
    for (int tile : {8, 16, 32})
        for (int waves : {4, 8, 16})
            for (int split : {4096, 8192, 16384})
                for (int sched : {1, 2})
                    for (int flush : {1, 2}) {
                        mw_tuning t{};
                        t.tile = tile;
                        t.wg_waves = waves;
                        t.split = split;
                        t.schedule = sched;
                        t.flush = flush;
                        t.order = 3;
                        t.variant = v4 ? 4 : (I.W * I.W <= 64 ? 1 : 3);
                        if (!v4 && sched == 2) continue;
                        if (v4 && tile == 32) continue;          // private 32x32 tiles: too few waves
                        if (!v4 && tile == 8) continue;
                        cands.push_back(t);
                    }
    float best_ms = 1e30f;
    Launch best = I.L;
    for (const mw_tuning &t : cands) {
        Launch L;
        if (!resolve_launch(I, &t, &L).ok()) continue; // does not fit LDS
        MWG_TRY(rebuild_schedule(I, L, s));
        float ms = 0.f;
        MWG_TRY(time_launch(I, (const float2 *)vis.p, (float2 *)grid.p, s, &ms));
        if (ms < best_ms) {
            best_ms = ms;
            best = L;
        }
    }
    MWG_TRY(rebuild_schedule(I, best, s));
    if (path) cache_store(path, key, best, best_ms);
    return Status::Ok();
}

} // namespace mwg
