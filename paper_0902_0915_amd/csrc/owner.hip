// Owner-tile schedule of the wave-tile gridder (flush 3).
//
// With flush 2 every work item grids its own tile's groups into a haloed LDS tile, writes
// the whole haloed tile to a scratch buffer, and a merge pass sums the up to nine tiles that
// cover each cell. For sparse instances (a few groups per tile) that scratch traffic, a
// haloed tile per handful of groups, dwarfs the visibilities themselves. Flush 3 turns the
// scatter into a gather by output tile: the plan lists, for every output tile, each sorted
// group whose footprint reaches it (from the tile and its neighbours), a wave grids that list
// into an LDS tile with a 2h margin and writes the tile's T x T cells once, and the output
// tiles no footprint reaches are written as zeros by a fill over their list. Each grid cell is
// written exactly once; the price is gridding the groups near a tile edge for each tile they
// reach (about 1.9 times the groups for T = 16 and W = 7).
//
// The lists are built on the device: per sorted group its output tiles (1, 2 or 4, since
// T >= W - 1), an exclusive scan of those counts, the (tile, sorted index) pairs, and a stable
// radix sort of the pairs by tile. Within a tile the candidates therefore keep the sorted
// order: by source tile, then cell and row sub-position, which the gridder's runs need.
#include "internal.h"
#include "gridder_core.h"

#include <algorithm>
#include <vector>

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

using Tmp = DevTmp;

// Output tiles [x0, x1] x [y0, y1] that the footprint of sorted group p reaches.
__device__ inline void reach(uint32_t p, int h, int lgT, int &x0, int &x1, int &y0, int &y1) {
    const int cx = (int)(p & 0xFFFu), cy = (int)((p >> 12) & 0xFFFu);
    x0 = (cx - h) >> lgT;
    x1 = (cx + h) >> lgT;
    y0 = (cy - h) >> lgT;
    y1 = (cy + h) >> lgT;
}

__global__ void k_owner_count(const uint32_t *spos, int64_t nk, int h, int lgT, uint32_t *count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nk) return;
    int x0, x1, y0, y1;
    reach(spos[i], h, lgT, x0, x1, y0, y1);
    count[i] = (uint32_t)((x1 - x0 + 1) * (y1 - y0 + 1));
}

__global__ void k_owner_emit(const uint32_t *spos, int64_t nk, int h, int lgT, int ntx, const uint32_t *offset,
                             uint32_t *keys, uint32_t *vals) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nk) return;
    int x0, x1, y0, y1;
    reach(spos[i], h, lgT, x0, x1, y0, y1);
    uint32_t o = offset[i];
    for (int ty = y0; ty <= y1; ty++)
        for (int tx = x0; tx <= x1; tx++) {
            keys[o] = (uint32_t)(ty * ntx + tx);
            vals[o] = (uint32_t)i;
            o++;
        }
}

__global__ void k_owner_bounds(const uint32_t *skeys, int64_t n, int32_t *tstart, int32_t *tend) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t t = skeys[i];
    if (i == 0 || skeys[i - 1] != t) tstart[t] = (int32_t)i;
    if (i == n - 1 || skeys[i + 1] != t) tend[t] = (int32_t)(i + 1);
}

// Per pair: the group's footprint origin in the output tile's LDS tile (origin 2h cells above
// and left of the tile, row stride R3) and its two tap-row offsets, as the gridder's codes.
__global__ void k_owner_codes(const uint32_t *skeys, const uint32_t *svals, int64_t n, const uint32_t *spos,
                              const uint32_t *perm, const float *sw, const uint32_t *sant, int T, int ntx, int h,
                              int R3, uint32_t *pcode, uint32_t *pperm, float *psw, uint32_t *psant) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const uint32_t o = skeys[k], i = svals[k];
    const uint32_t p = spos[i];
    const int cx = (int)(p & 0xFFFu), cy = (int)((p >> 12) & 0xFFFu);
    const uint32_t px = (p >> 24) & 0xFu, py = p >> 28;
    const int ox0 = (int)(o % (uint32_t)ntx) * T, oy0 = (int)(o / (uint32_t)ntx) * T;
    const uint32_t cell = (uint32_t)((cy - oy0 + h) * R3 + (cx - ox0 + h));
    pcode[k] = cell | ((px * 8u) << 16) | ((py * 8u) << 24);
    pperm[k] = perm[i];
    if (psw) psw[k] = sw[i];
    if (psant) psant[k] = sant[i];
}

template <int NPOL>
__global__ __launch_bounds__(256) void k_zero_tiles(float2 *grid, const int32_t *tiles, int n, int nx, int ny,
                                                    int T, int ntx) {
    const int wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    const int k = (int)blockIdx.x * 4 + wave;
    if (k >= n) return;
    const int t = tiles[k];
    zero_tile<NPOL>(grid, nx, ny, (t % ntx) * T, (t / ntx) * T, T, lane, 64);
}

} // namespace

Status build_owner_schedule(Instance &I, int64_t cap, bool *built, hipStream_t s) {
    *built = false;
    const int T = I.L.tile, lgT = ilog2(T), h = (I.W - 1) / 2;
    if (I.stacks || I.L.variant != 4) return make_error(MW_ERR_UNSUPPORTED, "flush 3 needs the wave-tile gridder");
    if (T < I.W - 1) return make_error(MW_ERR_UNSUPPORTED, "flush 3 needs tiles of at least W - 1 cells");
    const int ntx = (I.nx + T - 1) / T, nty = (I.ny + T - 1) / T;
    const int64_t ntiles = (int64_t)ntx * nty;
    const int64_t nk = I.nkept;
    if ((double)nk * 4.0 >= 4294967295.0)
        return make_error(MW_ERR_UNSUPPORTED, "flush 3 lists up to 2^32 (tile, group) pairs");
    std::vector<WorkItem> items;
    std::vector<int32_t> zero;
    int64_t npairs = 0;
    Tmp keys, keys2, vals, vals2, vinit, tstart, tend;
    uint32_t *sk = nullptr, *sv = nullptr;
    if (nk > 0) {
        Tmp counts;
        MWG_TRY(counts.alloc(4 * (size_t)(nk + 1), s));
        MWG_TRY(launch_fill_u32(counts.as<uint32_t>() + nk, 1, 0, s));
        hipLaunchKernelGGL(k_owner_count, dim3(grid1d(nk)), dim3(kBlock), 0, s, I.spos, nk, h, lgT,
                           counts.as<uint32_t>());
        MWG_HIP(hipGetLastError());
        MWG_TRY(exclusive_scan_u32(counts.as<uint32_t>(), nk + 1, s));
        uint32_t np = 0;
        MWG_HIP(hipMemcpyAsync(&np, counts.as<uint32_t>() + nk, 4, hipMemcpyDeviceToHost, s));
        MWG_HIP(hipStreamSynchronize(s));
        npairs = np;
        MWG_TRY(keys.alloc(4 * (size_t)npairs, s));
        MWG_TRY(keys2.alloc(4 * (size_t)npairs, s));
        MWG_TRY(vals.alloc(4 * (size_t)npairs, s));
        MWG_TRY(vals2.alloc(4 * (size_t)npairs, s));
        MWG_TRY(vinit.alloc(4 * (size_t)npairs, s));
        hipLaunchKernelGGL(k_owner_emit, dim3(grid1d(nk)), dim3(kBlock), 0, s, I.spos, nk, h, lgT, ntx,
                           counts.as<uint32_t>(), keys.as<uint32_t>(), vinit.as<uint32_t>());
        MWG_HIP(hipGetLastError());
        MWG_TRY(sort_pairs(keys.as<uint32_t>(), keys2.as<uint32_t>(), vinit.as<uint32_t>(), vals.as<uint32_t>(),
                           vals2.as<uint32_t>(), npairs, std::max(1, bitlen((uint64_t)ntiles)), &sk, &sv, s));
        MWG_TRY(tstart.alloc(4 * (size_t)ntiles, s));
        MWG_TRY(tend.alloc(4 * (size_t)ntiles, s));
        MWG_TRY(launch_fill_u32(tstart.as<uint32_t>(), ntiles, 0, s));
        MWG_TRY(launch_fill_u32(tend.as<uint32_t>(), ntiles, 0, s));
        hipLaunchKernelGGL(k_owner_bounds, dim3(grid1d(npairs)), dim3(kBlock), 0, s, sk, npairs, tstart.as<int32_t>(),
                           tend.as<int32_t>());
        MWG_HIP(hipGetLastError());
    }
    std::vector<int32_t> hs((size_t)ntiles, 0), he((size_t)ntiles, 0);
    if (nk > 0) {
        MWG_HIP(hipMemcpyAsync(hs.data(), tstart.p, 4 * ntiles, hipMemcpyDeviceToHost, s));
        MWG_HIP(hipMemcpyAsync(he.data(), tend.p, 4 * ntiles, hipMemcpyDeviceToHost, s));
        MWG_HIP(hipStreamSynchronize(s));
    }
    int maxn = 0;
    for (int64_t t = 0; t < ntiles; t++) {
        const int cnt = he[t] - hs[t];
        if (cnt > 0) {
            items.push_back({(int32_t)t, hs[t], he[t], 0});
            maxn = std::max(maxn, cnt);
        } else {
            zero.push_back((int32_t)t);
        }
    }
    if (cap > 0 && maxn > cap) return Status::Ok();  // too dense: the caller keeps flush 2
    // largest first, ties in tile order
    std::stable_sort(items.begin(), items.end(),
                     [](const WorkItem &a, const WorkItem &b) { return a.end - a.begin > b.end - b.begin; });
    void *p;
    if (I.cap_pairs < (size_t)std::max<int64_t>(npairs, 1)) {
        I.cap_pairs = (size_t)std::max<int64_t>(npairs, 1);
        MWG_TRY(I.arena.alloc(&p, 4 * I.cap_pairs));
        I.pperm = (uint32_t *)p;
        MWG_TRY(I.arena.alloc(&p, 4 * I.cap_pairs));
        I.pcode = (uint32_t *)p;
        if (I.sw) {
            MWG_TRY(I.arena.alloc(&p, 4 * I.cap_pairs));
            I.psw = (float *)p;
        }
        if (I.sant) {
            MWG_TRY(I.arena.alloc(&p, 4 * I.cap_pairs));
            I.psant = (uint32_t *)p;
        }
    }
    if (I.cap_owork < std::max<size_t>(items.size(), 1)) {
        I.cap_owork = std::max<size_t>(items.size(), 1);
        MWG_TRY(I.arena.alloc(&p, sizeof(WorkItem) * I.cap_owork));
        I.owork = (WorkItem *)p;
    }
    if (I.cap_ozero < std::max<size_t>(zero.size(), 1)) {
        I.cap_ozero = std::max<size_t>(zero.size(), 1);
        MWG_TRY(I.arena.alloc(&p, 4 * I.cap_ozero));
        I.ozero = (int32_t *)p;
    }
    if (npairs > 0) {
        hipLaunchKernelGGL(k_owner_codes, dim3(grid1d(npairs)), dim3(kBlock), 0, s, sk, sv, npairs, I.spos, I.perm,
                           I.sw, I.sant, T, ntx, h, owner_span(T, I.W), I.pcode, I.pperm, I.sw ? I.psw : nullptr,
                           I.sant ? I.psant : nullptr);
        MWG_HIP(hipGetLastError());
    }
    // the host lists stay in the instance (the uploads are not waited for here)
    I.h_owork.swap(items);
    I.h_ozero.swap(zero);
    if (!I.h_owork.empty())
        MWG_HIP(hipMemcpyAsync(I.owork, I.h_owork.data(), sizeof(WorkItem) * I.h_owork.size(), hipMemcpyHostToDevice,
                               s));
    if (!I.h_ozero.empty())
        MWG_HIP(hipMemcpyAsync(I.ozero, I.h_ozero.data(), 4 * I.h_ozero.size(), hipMemcpyHostToDevice, s));
    I.owner_tile = T;
    I.nowork = (int)I.h_owork.size();
    I.n_ozero = (int)I.h_ozero.size();
    I.max_owner_groups = maxn;
    I.npairs_owner = npairs;
    *built = true;
    return Status::Ok();
}

Status launch_zero_tiles(const Instance &I, float2 *grid, hipStream_t s) {
    if (I.n_ozero <= 0) return Status::Ok();
    const dim3 g((unsigned)((I.n_ozero + 3) / 4)), b(256);
    const int T = I.owner_tile;
    switch (I.npol) {
    case 1: hipLaunchKernelGGL(k_zero_tiles<1>, g, b, 0, s, grid, I.ozero, I.n_ozero, I.nx, I.ny, T, I.ntx); break;
    case 2: hipLaunchKernelGGL(k_zero_tiles<2>, g, b, 0, s, grid, I.ozero, I.n_ozero, I.nx, I.ny, T, I.ntx); break;
    case 4: hipLaunchKernelGGL(k_zero_tiles<4>, g, b, 0, s, grid, I.ozero, I.n_ozero, I.nx, I.ny, T, I.ntx); break;
    default: return make_error(MW_ERR_UNSUPPORTED, "npol %d", I.npol);
    }
    MWG_HIP(hipGetLastError());
    return Status::Ok();
}

} // namespace mwg
