// The block-padded work list of gridder variant 6: the plan's sorted groups with every run of
// equal (cell, py) inside a work item padded to a multiple of kRunBlock entries, so that the
// gridder takes each block of kRunBlock entries as one run without a test per group.
//
// From the current sort (spos, perm, scode and the optional sw, sant, all in sorted order)
// and the work items (which partition the sorted range): a run starts at an item's first
// entry and wherever (cell, py) changes; a scan numbers the runs; each run's length is
// rounded up to a multiple of kRunBlock; a second scan places the runs; the entries are
// scattered to their padded positions and each run's padding entries are written as
// kDummyGroup with the run's code (the gridder stages them as zero visibilities); the
// items' ranges are moved to the padded positions. One synchronisation, for the padded size.
#include "internal.h"
#include "gridder_core.h"

#include <algorithm>

namespace mwg {

Status exclusive_scan_u32(uint32_t *data, int64_t n, hipStream_t s);
Status launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);

namespace {

constexpr int kBlock = 256;

unsigned grid1d(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// the (cell, py) of a packed position, without px
__device__ inline uint32_t run_key(uint32_t p) { return p & 0xF0FFFFFFu; }

__global__ void k_item_starts(const WorkItem *work, int nwork, uint32_t *flag) {
    const int w = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (w < nwork && work[w].end > work[w].begin) flag[work[w].begin] = 1u;
}

__global__ void k_run_flags(const uint32_t *spos, int64_t n, uint32_t *flag, uint32_t *copy) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t f = flag[i];
    if (i == 0 || run_key(spos[i]) != run_key(spos[i - 1])) f = 1u;
    flag[i] = f;
    copy[i] = f;
}

// run of entry i from the exclusive scan of the flags
__device__ inline uint32_t run_of(const uint32_t *scan, const uint32_t *flag, int64_t i) {
    return scan[i] + flag[i] - 1u;
}

__global__ void k_run_first(const uint32_t *flag, const uint32_t *scan, int64_t n, uint32_t *first) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && flag[i]) first[scan[i]] = (uint32_t)i;
}

// padded length of every run (runs past the last are empty); nruns from the scan's end
__global__ void k_run_padded(const uint32_t *first, const uint32_t *flag, const uint32_t *scan, int64_t n,
                             uint32_t *plen) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r > n) return;
    const uint32_t nruns = scan[n - 1] + flag[n - 1];
    uint32_t len = 0;
    if (r < nruns) {
        const uint32_t next = (r + 1 < nruns) ? first[r + 1] : (uint32_t)n;
        len = next - first[r];
    }
    plen[r] = (len + (uint32_t)(kRunBlock - 1)) & ~(uint32_t)(kRunBlock - 1);
}

__global__ void k_run_scatter(const uint32_t *flag, const uint32_t *scan, const uint32_t *first,
                              const uint32_t *pstart, int64_t n, const uint32_t *perm, const uint32_t *scode,
                              const float *sw, const uint32_t *sant, uint32_t *bperm, uint32_t *bcode, float *bsw,
                              uint32_t *bsant) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t r = run_of(scan, flag, i);
    const uint32_t pos = pstart[r] + ((uint32_t)i - first[r]);
    bperm[pos] = perm[i];
    bcode[pos] = scode[i];
    if (bsw) bsw[pos] = sw[i];
    if (bsant) bsant[pos] = sant[i];
}

// the padding entries of every run
__global__ void k_run_pad(const uint32_t *first, const uint32_t *flag, const uint32_t *scan, const uint32_t *pstart,
                          int64_t n, const uint32_t *scode, uint32_t *bperm, uint32_t *bcode, float *bsw,
                          uint32_t *bsant) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nruns = scan[n - 1] + flag[n - 1];
    if (r >= nruns) return;
    const uint32_t next = (r + 1 < nruns) ? first[r + 1] : (uint32_t)n;
    const uint32_t len = next - first[r];
    const uint32_t code = scode[first[r]];
    for (uint32_t k = len; k < pstart[r + 1] - pstart[r]; k++) {
        const uint32_t pos = pstart[r] + k;
        bperm[pos] = kDummyGroup;
        bcode[pos] = code;
        if (bsw) bsw[pos] = 0.0f;
        if (bsant) bsant[pos] = 0u;
    }
}

// read-ahead entries past the end of the padded list
__global__ void k_run_tail(uint32_t *bperm, uint32_t *bcode, const uint32_t *pstart, int64_t n) {
    const uint32_t end = pstart[n];
    bperm[end + threadIdx.x] = kDummyGroup;
    bcode[end + threadIdx.x] = 0u;
}

__global__ void k_run_items(const WorkItem *work, int nwork, const uint32_t *flag, const uint32_t *scan,
                            const uint32_t *pstart, WorkItem *bwork) {
    const int w = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (w >= nwork) return;
    WorkItem wk = work[w];
    if (wk.end > wk.begin) {
        const uint32_t r0 = run_of(scan, flag, wk.begin), r1 = run_of(scan, flag, wk.end - 1);
        wk.begin = (int32_t)pstart[r0];
        wk.end = (int32_t)pstart[r1 + 1];
    } else {
        wk.begin = wk.end = 0;
    }
    bwork[w] = wk;
}

} // namespace

Status build_block_schedule(Instance &I, hipStream_t s) {
    const int64_t nk = I.nkept;
    void *p;
    if (I.cap_bwork < std::max<size_t>((size_t)I.nwork, 1)) {  // as many items as the sorted list
        I.cap_bwork = std::max<size_t>((size_t)I.nwork, 1);
        MWG_TRY(I.arena.alloc(&p, sizeof(WorkItem) * I.cap_bwork));
        I.bwork = (WorkItem *)p;
    }
    if (nk == 0 || I.nwork == 0) {
        I.nblocked = 0;
        I.block_tile = I.L.tile;
        if (!I.bperm) {
            MWG_TRY(I.arena.alloc(&p, 4 * 64));
            I.bperm = (uint32_t *)p;
            MWG_TRY(I.arena.alloc(&p, 4 * 64));
            I.bcode = (uint32_t *)p;
        }
        return Status::Ok();
    }
    DevTmp flag, scan, first, plen;
    MWG_TRY(flag.alloc(4 * (size_t)nk, s));
    MWG_TRY(scan.alloc(4 * (size_t)nk, s));
    MWG_TRY(first.alloc(4 * (size_t)nk, s));
    MWG_TRY(plen.alloc(4 * ((size_t)nk + 1), s));
    MWG_TRY(launch_fill_u32(flag.as<uint32_t>(), nk, 0u, s));
    hipLaunchKernelGGL(k_item_starts, dim3(grid1d(I.nwork)), dim3(kBlock), 0, s, I.work, I.nwork,
                       flag.as<uint32_t>());
    hipLaunchKernelGGL(k_run_flags, dim3(grid1d(nk)), dim3(kBlock), 0, s, I.spos, nk, flag.as<uint32_t>(),
                       scan.as<uint32_t>());
    MWG_HIP(hipGetLastError());
    MWG_TRY(exclusive_scan_u32(scan.as<uint32_t>(), nk, s));
    hipLaunchKernelGGL(k_run_first, dim3(grid1d(nk)), dim3(kBlock), 0, s, flag.as<uint32_t>(),
                       scan.as<uint32_t>(), nk, first.as<uint32_t>());
    hipLaunchKernelGGL(k_run_padded, dim3(grid1d(nk + 1)), dim3(kBlock), 0, s, first.as<uint32_t>(),
                       flag.as<uint32_t>(), scan.as<uint32_t>(), nk, plen.as<uint32_t>());
    MWG_HIP(hipGetLastError());
    MWG_TRY(exclusive_scan_u32(plen.as<uint32_t>(), nk + 1, s));  // run starts; total at [nk]
    uint32_t npad = 0;
    MWG_HIP(hipMemcpyAsync(&npad, plen.as<uint32_t>() + nk, 4, hipMemcpyDeviceToHost, s));
    MWG_HIP(hipStreamSynchronize(s));
    if ((int64_t)npad > ((int64_t)1 << 31) - 64)
        return make_error(MW_ERR_UNSUPPORTED, "the padded work list exceeds 2^31 entries");
    if (I.cap_blocked < (int64_t)npad) {
        I.cap_blocked = npad;
        MWG_TRY(I.arena.alloc(&p, 4 * ((size_t)npad + 64)));
        I.bperm = (uint32_t *)p;
        MWG_TRY(I.arena.alloc(&p, 4 * ((size_t)npad + 64)));
        I.bcode = (uint32_t *)p;
        if (I.sw) {
            MWG_TRY(I.arena.alloc(&p, 4 * (size_t)npad));
            I.bsw = (float *)p;
        }
        if (I.sant) {
            MWG_TRY(I.arena.alloc(&p, 4 * (size_t)npad));
            I.bsant = (uint32_t *)p;
        }
    }
    hipLaunchKernelGGL(k_run_scatter, dim3(grid1d(nk)), dim3(kBlock), 0, s, flag.as<uint32_t>(), scan.as<uint32_t>(),
                       first.as<uint32_t>(), plen.as<uint32_t>(), nk, I.perm, I.scode, I.sw, I.sant, I.bperm,
                       I.bcode, I.sw ? I.bsw : nullptr, I.sant ? I.bsant : nullptr);
    hipLaunchKernelGGL(k_run_pad, dim3(grid1d(nk)), dim3(kBlock), 0, s, first.as<uint32_t>(), flag.as<uint32_t>(),
                       scan.as<uint32_t>(), plen.as<uint32_t>(), nk, I.scode, I.bperm, I.bcode,
                       I.sw ? I.bsw : nullptr, I.sant ? I.bsant : nullptr);
    hipLaunchKernelGGL(k_run_tail, dim3(1), dim3(64), 0, s, I.bperm, I.bcode, plen.as<uint32_t>(), nk);
    hipLaunchKernelGGL(k_run_items, dim3(grid1d(I.nwork)), dim3(kBlock), 0, s, I.work, I.nwork,
                       flag.as<uint32_t>(), scan.as<uint32_t>(), plen.as<uint32_t>(), I.bwork);
    MWG_HIP(hipGetLastError());
    I.nblocked = npad;
    I.block_tile = I.L.tile;
    return Status::Ok();
}

} // namespace mwg
