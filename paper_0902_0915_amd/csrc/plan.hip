// Plan construction: FP64 positions and quantisation, the keep rule, the stable radix sort
// by uv tile (and cell), tile bounds, the heavy-tile split into work items, and the
// kernel tables.
//
// The paper says the GPU port needed new memory structures and some algorithmic changes to
// suit the hardware's access-pattern sensitivity (Section 3.2). Here that is the plan: the
// visibilities' positions never change between calls, so they are computed, quantised and
// sorted by grid tile once, and every later grid/degrid call walks the sorted order.
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

namespace mwg {

Status make_error(mw_status code, const char *fmt, ...) {
    Status s;
    s.code = code;
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    s.msg = buf;
    return s;
}

// Arrays of less than kArenaSmall bytes are carved, 256-byte aligned, from chunks of
// kArenaChunk bytes: a plan owns dozens of small arrays (work lists, tables, per-antenna
// buffers), and one hipMalloc each would dominate the time to build plans of small instances.
constexpr size_t kArenaSmall = size_t(256) << 10;
constexpr size_t kArenaChunk = size_t(2) << 20;

Status DevArena::alloc(void **p, size_t nbytes) {
    *p = nullptr;
    if (nbytes == 0) nbytes = 16;
    nbytes = (nbytes + 255) & ~size_t(255);
    if (nbytes < kArenaSmall && nbytes <= chunk_left) {
        *p = chunk;
        chunk += nbytes;
        chunk_left -= nbytes;
        bytes += (int64_t)nbytes;
        return Status::Ok();
    }
    const size_t take = nbytes < kArenaSmall ? kArenaChunk : nbytes;
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, take);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return make_error(MW_ERR_ALLOC, "hipMalloc(%zu) failed: %s", take, hipGetErrorString(e));
    }
    ptrs.push_back(q);
    if (nbytes < kArenaSmall) {  // a new chunk: the rest of it serves later small arrays
        chunk = (char *)q + nbytes;
        chunk_left = take - nbytes;
    }
    *p = q;
    bytes += (int64_t)nbytes;
    return Status::Ok();
}

void DevArena::release() {
    for (void *p : ptrs) (void)hipFree(p);
    ptrs.clear();
    bytes = 0;
    chunk = nullptr;
    chunk_left = 0;
}

// Blocks of the temporary pool grow geometrically from kTmpBlock bytes; a block, once
// allocated, lives until its scope ends. Allocations form a stack: a record is popped when it
// and every record above it have been given back, and the top of its block falls back to it.
constexpr size_t kTmpBlock = size_t(16) << 20;

struct TmpPool {
    struct Block {
        char *base;
        size_t size, top;
    };
    struct Rec {
        void *p;
        int block;
        size_t off;
        bool freed;
    };
    hipStream_t stream = nullptr;
    size_t first = 0;  // size of the first block (0: kTmpBlock)
    std::vector<Block> blocks;
    std::vector<Rec> stack;

    Status take(size_t nbytes, void **out) {
        nbytes = (nbytes + 255) & ~size_t(255);
        int b = stack.empty() ? 0 : stack.back().block;  // blocks after b are empty
        while (b < (int)blocks.size() && blocks[b].size - blocks[b].top < nbytes) b++;
        if (b == (int)blocks.size()) {
            size_t want = blocks.empty() ? std::max(kTmpBlock, first) : kTmpBlock;
            for (const Block &k : blocks) want = std::max(want, 2 * k.size);
            want = std::max(want, nbytes);
            void *q = nullptr;
            hipError_t e = hipMalloc(&q, want);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                return make_error(MW_ERR_ALLOC, "hipMalloc(%zu) failed: %s", want, hipGetErrorString(e));
            }
            blocks.push_back({(char *)q, want, 0});
        }
        Block &k = blocks[b];
        *out = k.base + k.top;
        stack.push_back({*out, b, k.top, false});
        k.top += nbytes;
        return Status::Ok();
    }
    void give_back(void *p) {
        for (size_t i = stack.size(); i-- > 0;)
            if (stack[i].p == p && !stack[i].freed) {
                stack[i].freed = true;
                break;
            }
        while (!stack.empty() && stack.back().freed) {
            blocks[stack.back().block].top = stack.back().off;
            stack.pop_back();
        }
    }
};

namespace {
thread_local TmpPool *t_tmp_pool = nullptr;
}

Status DevTmp::alloc(size_t nbytes, hipStream_t s) {
    release();
    if (nbytes == 0) nbytes = 16;
    if (t_tmp_pool && t_tmp_pool->stream == s) {
        MWG_TRY(t_tmp_pool->take(nbytes, &p));
        pool = t_tmp_pool;
        return Status::Ok();
    }
    hipError_t e = hipMalloc(&p, nbytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
        return make_error(MW_ERR_ALLOC, "hipMalloc(%zu) failed: %s", nbytes, hipGetErrorString(e));
    }
    return Status::Ok();
}

void DevTmp::release() {
    if (!p) return;
    if (pool)
        pool->give_back(p);
    else
        (void)hipFree(p);
    p = nullptr;
    pool = nullptr;
}

TmpScope::TmpScope(hipStream_t s, size_t first_block) {
    if (t_tmp_pool) return;
    own = new TmpPool();
    own->stream = s;
    own->first = first_block;
    t_tmp_pool = own;
}

size_t plan_tmp_hint(int64_t ngroups, int nx, int ny) {
    return 17 * (size_t)std::max<int64_t>(ngroups, 0) + 2 * (size_t)nx * (size_t)ny + (size_t(4) << 20);
}

TmpScope::~TmpScope() {
    if (!own) return;
    t_tmp_pool = nullptr;
    // no queued kernel may still read a block when it is freed
    (void)hipStreamSynchronize(own->stream);
    for (const TmpPool::Block &k : own->blocks) (void)hipFree(k.base);
    delete own;
}

namespace {

constexpr int kBlock = 256;

using Tmp = DevTmp;

// ------------------------------------------------------------------------------------------
// A1: positions. One thread per group; every operation rounded to FP64 in the stated order
// (no contraction), so the integers agree bit for bit with any IEEE FP64 evaluation of the
// same rule.
// ------------------------------------------------------------------------------------------
struct PosArgs {
    int64_t ngroups;
    int nchan, nx, ny, O, h;
    double du, dv;
    const double *uvw, *freq;
    const uint8_t *flags;
    const float *weights;
    const int32_t *kidx;   // stacks: kernel of each group
    const int32_t *ksup;   // stacks: support of each kernel
    uint32_t *pos;
    uint32_t *blk_counts;  // [gridDim.x][3]: kept, flagged, outside of each block
    int wsel;              // keep only wlo <= w < whi (one plane of w-stacking)
    double wlo, whi;
};

__global__ void k_positions(PosArgs a) {
#pragma clang fp contract(off)
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int status = 3; // 0 kept, 1 flagged, 2 outside, 3 out of range
    if (g < a.ngroups) {
        uint32_t packed = kDropped;
        // 32-bit integer work throughout: groups < 2^31 (checked when the plan is built)
        const uint32_t g32 = (uint32_t)g, nc = (uint32_t)a.nchan;
        const int64_t r = (int64_t)(g32 / nc);
        const int ch = (int)(g32 - (uint32_t)r * nc);
        const double f = a.freq[ch];
        bool deselected = false;
        if (a.wsel) {
            const double w = (a.uvw[3 * r + 2] * f) / 299792458.0;
            deselected = !(w >= a.wlo && w < a.whi);
        }
        if ((a.flags && a.flags[g]) || (a.weights && a.weights[g] == 0.0f) || deselected) {
            status = 1;
        } else {
            const double u = (a.uvw[3 * r + 0] * f) / 299792458.0;
            const double v = (a.uvw[3 * r + 1] * f) / 299792458.0;
            const double x = u / a.du + (double)(a.nx / 2);
            const double y = v / a.dv + (double)(a.ny / 2);
            const double qxd = floor(x * (double)a.O + 0.5);
            const double qyd = floor(y * (double)a.O + 0.5);
            status = 2;
            // |q| >= 2^24 puts the cell more than 2^20 - 1 cells from the centre (O <= 16),
            // outside any grid of at most 4096 cells: such groups (and NaN) are outside
            // without the integer steps, which then fit 32 bits
            if (fabs(qxd) < 16777216.0 && fabs(qyd) < 16777216.0) {
                const int qx = (int)qxd, qy = (int)qyd;
                const int half = a.O / 2;
                int cx = (qx + half) / a.O, cy = (qy + half) / a.O;
                if ((qx + half) % a.O != 0 && (qx + half) < 0) cx -= 1; // floor division
                if ((qy + half) % a.O != 0 && (qy + half) < 0) cy -= 1;
                const int px = qx - cx * a.O, py = qy - cy * a.O;
                const int h = a.kidx ? (a.ksup[a.kidx[g]] - 1) / 2 : a.h;
                if (cx - h >= 0 && cx + h < a.nx && cy - h >= 0 && cy + h < a.ny) {
                    packed = pack_pos((int)cx, (int)cy, (int)(px + half), (int)(py + half));
                    status = 0;
                }
            }
        }
        a.pos[g] = packed;
    }
    // Counts per block, no atomics: every wave stores its three ballot counts in LDS, the
    // first thread sums them and writes the block's entry (a later kernel sums the blocks).
    // Atomics from every wave on one counter serialise the waves.
    __shared__ uint32_t wc[kBlock / 64][3];
    const unsigned long long k0 = __ballot(status == 0), k1 = __ballot(status == 1),
                             k2 = __ballot(status == 2);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        wc[w][0] = (uint32_t)__popcll(k0);
        wc[w][1] = (uint32_t)__popcll(k1);
        wc[w][2] = (uint32_t)__popcll(k2);
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        uint32_t t = 0;
        for (int k = 0; k < kBlock / 64; k++) t += wc[k][threadIdx.x];
        a.blk_counts[(int64_t)blockIdx.x * 3 + threadIdx.x] = t;
    }
}

// Sums the per-block counts: out[c] += sum over blocks of cnt[b][c] (out zeroed before),
// a grid-stride sum per workgroup and three atomics per workgroup.
constexpr int kSumBlocks = 128;
__global__ void k_sum_counts(const uint32_t *cnt, int64_t nblocks, unsigned long long *out) {
    __shared__ unsigned long long part[kBlock / 64][3];
    unsigned long long t[3] = {0, 0, 0};
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nblocks; b += (int64_t)gridDim.x * blockDim.x)
        for (int c = 0; c < 3; c++) t[c] += cnt[b * 3 + c];
    for (int c = 0; c < 3; c++) {
        unsigned long long v = t[c];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
        if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6][c] = v;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        unsigned long long v = 0;
        for (int k = 0; k < kBlock / 64; k++) v += part[k][threadIdx.x];
        if (v) atomicAdd(&out[threadIdx.x], v);
    }
}

// Occupied 8 x 8 tiles: one bit per tile, set by the first group found in it (a group that
// sees its bit already set issues no atomic), then a population count. A batched plan picks its
// tile size from this count before any schedule is built.
constexpr int kCountTile = 8;

__global__ void k_mark_tiles(const uint32_t *pos, int64_t n, int ntx, uint32_t *bits) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const uint32_t p = pos[g];
    if (p == kDropped) return;
    const int t = (int)(((p >> 12) & 0xFFFu) / kCountTile) * ntx + (int)((p & 0xFFFu) / kCountTile);
    uint32_t *w = bits + (t >> 5);
    const uint32_t m = 1u << (t & 31);
    if (!(__atomic_load_n(w, __ATOMIC_RELAXED) & m)) atomicOr(w, m);
}

__global__ void k_popcount(const uint32_t *bits, int64_t nwords, unsigned long long *out) {
    __shared__ unsigned long long part[kBlock / 64];
    unsigned long long v = 0;
    for (int64_t i = threadIdx.x; i < nwords; i += blockDim.x) v += (unsigned long long)__popc(bits[i]);
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0;
        for (int k = 0; k < kBlock / 64; k++) s += part[k];
        *out = s;
    }
}

// Sort keys: tile-major, then cell within the tile (order 1) or nothing (order 2: the stable
// sort keeps input order). Dropped groups get the all-ones key of the sorted width.
// Rank of cell (cx, cy) among the cells of its tile ordered by their line across the radius
// (the direction from the grid centre to the tile centre), then by their position along it,
// then by cell index. Integer arithmetic on cell-centre offsets doubled and a direction scaled
// to 2^10, so that every comparison is exact and the ranks are a permutation of the tile's
// cells. Tiles above 16 x 16 keep rows in tiles that lie more in u than in v, and columns
// otherwise.
__device__ inline uint32_t radial_rank(uint32_t cx, uint32_t cy, int tb, int nx, int ny) {
    const int T = 1 << tb, mask = T - 1;
    const int lx = (int)(cx & (uint32_t)mask), ly = (int)(cy & (uint32_t)mask);
    const int du = (int)((cx >> tb) << tb) + T / 2 - nx / 2;
    const int dv = (int)((cy >> tb) << tb) + T / 2 - ny / 2;
    if (tb > 4)
        return abs(dv) > abs(du) ? (uint32_t)((lx << tb) | ly) : (uint32_t)((ly << tb) | lx);
    const float len = sqrtf((float)du * (float)du + (float)dv * (float)dv);
    const int ex = len > 0.0f ? (int)lrintf(1024.0f * (float)du / len) : 1024;
    const int ey = len > 0.0f ? (int)lrintf(1024.0f * (float)dv / len) : 0;
    // line index: the cross-radial coordinate in cells, rounded (units of 1/2048 cell);
    // position: the radial coordinate (same units)
    auto line = [&](int x, int y) {
        const int v = -ey * (2 * x - (T - 1)) + ex * (2 * y - (T - 1));
        return (v + 1024 + (64 << 11)) >> 11;  // floor((v + 1024) / 2048) + 64, non-negative
    };
    auto along = [&](int x, int y) { return ex * (2 * x - (T - 1)) + ey * (2 * y - (T - 1)); };
    const int l0 = line(lx, ly), a0 = along(lx, ly), i0 = ly * T + lx;
    uint32_t rank = 0;
    for (int y = 0; y < T; y++)
        for (int x = 0; x < T; x++) {
            const int l = line(x, y), a = along(x, y), i = y * T + x;
            rank += (l < l0 || (l == l0 && (a < a0 || (a == a0 && i < i0)))) ? 1u : 0u;
        }
    return rank;
}

// radial_rank of every cell of every tile, tile-major (T <= 16, so a rank fits a byte): for
// plans with more groups than cells, computed once per cell instead of once per group.
__global__ void k_rank_table(int tb, int ntx, int64_t ncells, int nx, int ny, uint8_t *ranks) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ncells) return;
    const int64_t tile = g >> (2 * tb);
    const uint32_t c = (uint32_t)(g & ((1 << (2 * tb)) - 1)), mask = (1u << tb) - 1u;
    const uint32_t cx = ((uint32_t)(tile % ntx) << tb) | (c & mask), cy = ((uint32_t)(tile / ntx) << tb) | (c >> tb);
    ranks[g] = (uint8_t)radial_rank(cx, cy, tb, nx, ny);
}

__global__ void k_keys(const uint32_t *pos, int64_t n, int tb, int ntx, int nx, int ny, int order,
                       uint32_t sentinel, const uint8_t *ranks, uint32_t *keys) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const uint32_t p = pos[g];
    uint32_t k = sentinel;
    if (p != kDropped) {
        const uint32_t cx = p & 0xFFFu, cy = (p >> 12) & 0xFFFu;
        const uint32_t tile = (cy >> tb) * (uint32_t)ntx + (cx >> tb);
        const uint32_t mask = (1u << tb) - 1u;
        if (order == 2) {
            k = tile;
        } else {
            // order 1: (tile, cell row, cell column, row sub-position). Order 3 replaces the
            // cell's (row, column) by its rank along the tile's radial direction: the channels
            // of one baseline fall on radially neighbouring cells, which this makes
            // consecutive.
            uint32_t cell = ((cy & mask) << tb) | (cx & mask);
            if (order == 3) cell = ranks ? (uint32_t)ranks[((size_t)tile << (2 * tb)) | cell] : radial_rank(cx, cy, tb, nx, ny);
            k = (tile << (2 * tb + 4)) | (cell << 4) | (p >> 28);
        }
    }
    keys[g] = k;
}

// ------------------------------------------------------------------------------------------
// A2: stable LSD radix sort of (key, index) pairs, 8 bits per pass.
//   hist:    per block digit counts, stored digit-major [256][nblocks]
//   scan:    exclusive prefix over that array -> each (digit, block) output base
//   scatter: each block ranks its keys stably (wave ballots for equal digits, waves in
//            order), places them in LDS in digit order, then writes each digit's run to
//            consecutive positions from its output base.
// ------------------------------------------------------------------------------------------
constexpr int kSortItems = 16;                 // keys per thread per block
constexpr int kSortChunk = kBlock * kSortItems; // keys per block

__global__ void k_rs_hist(const uint32_t *keys, int64_t n, int shift, uint32_t *hist, int nblocks) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortChunk;
    for (int it = 0; it < kSortItems; it++) {
        const int64_t i = base + (int64_t)it * kBlock + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kBlock) void k_rs_scatter(const uint32_t *keys_in, const uint32_t *vals_in,
                                                     uint32_t *keys_out, uint32_t *vals_out,
                                                     const uint32_t *offsets, int64_t n, int shift, int nblocks) {
    __shared__ uint32_t gbase[256], lstart[256], run[256], wsum[kBlock / 64];
    __shared__ uint32_t wcnt[kBlock / 64][256];
    __shared__ uint32_t stk[kSortChunk], stv[kSortChunk];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // this block's count of digit tid, from the scanned digit-major (digit, block) array
    const int64_t idx = (int64_t)tid * nblocks + blockIdx.x;
    const uint32_t off = offsets[idx];
    const uint32_t cnt = (idx + 1 < (int64_t)256 * nblocks ? offsets[idx + 1] : (uint32_t)n) - off;
    uint32_t inc = cnt;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    uint32_t wb = 0;
    for (int w = 0; w < wave; w++) wb += wsum[w];
    gbase[tid] = off;
    lstart[tid] = wb + inc - cnt;
    run[tid] = wb + inc - cnt;
    for (int w = 0; w < kBlock / 64; w++) wcnt[w][tid] = 0;
    __syncthreads();
    // stable ranks within the block (items in order, waves in order, lanes in order): each
    // key is placed in LDS at its digit's local start plus its rank
    const int64_t base = (int64_t)blockIdx.x * kSortChunk;
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int it = 0; it < kSortItems; it++) {
        const int64_t i = base + (int64_t)it * kBlock + tid;
        const bool valid = i < n;
        const uint32_t k = valid ? keys_in[i] : 0u;
        const uint32_t v = valid ? (vals_in ? vals_in[i] : (uint32_t)i) : 0u;
        const uint32_t d = (k >> shift) & 255u;
        unsigned long long peers = __ballot(valid);
        for (int b = 0; b < 8; b++) {
            const bool bit = (d >> b) & 1u;
            const unsigned long long m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const int rank = __popcll(peers & below);
        if (valid && rank == 0) wcnt[wave][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = run[d] + (uint32_t)rank;
            for (int w = 0; w < wave; w++) pos += wcnt[w][d];
            stk[pos] = k;
            stv[pos] = v;
        }
        __syncthreads();
        uint32_t tot = 0;
        for (int w = 0; w < kBlock / 64; w++) {
            tot += wcnt[w][tid];
            wcnt[w][tid] = 0;
        }
        run[tid] += tot;
        __syncthreads();
    }
    // the staged keys in digit order: each digit's run goes to consecutive global positions
    const int nvalid = (int)((n - base) < kSortChunk ? (n - base) : kSortChunk);
    for (int j = tid; j < nvalid; j += kBlock) {
        const uint32_t k = stk[j], d = (k >> shift) & 255u;
        const uint32_t g = gbase[d] + ((uint32_t)j - lstart[d]);
        keys_out[g] = k;
        vals_out[g] = stv[j];
    }
}

// Exclusive scan of uint32 (totals < 2^32): 1024 items per block, block sums scanned
// recursively, then added back.
constexpr int kScanItems = 4;
constexpr int kScanChunk = kBlock * kScanItems;

__global__ void k_scan_block(uint32_t *data, int64_t n, uint32_t *sums) {
    __shared__ uint32_t wsum[kBlock / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)tid * kScanItems;
    uint32_t v[kScanItems], t = 0;
    for (int j = 0; j < kScanItems; j++) {
        v[j] = (base + j < n) ? data[base + j] : 0u;
        t += v[j];
    }
    // inclusive scan of t across the wave
    uint32_t inc = t;
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    uint32_t wbase = 0;
    for (int w = 0; w < wave; w++) wbase += wsum[w];
    uint32_t run = wbase + inc - t;
    for (int j = 0; j < kScanItems; j++) {
        if (base + j < n) data[base + j] = run;
        run += v[j];
    }
    if (tid == kBlock - 1) sums[blockIdx.x] = wbase + inc;
}

__global__ void k_scan_add(uint32_t *data, int64_t n, const uint32_t *sums) {
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
    const uint32_t add = sums[blockIdx.x];
    for (int j = 0; j < kScanItems; j++)
        if (base + j < n) data[base + j] += add;
}

// Words of scratch scan_exclusive needs for n items: one partial sum per block at every
// level of the recursion.
int64_t scan_ws_words(int64_t n) {
    int64_t w = 0;
    while (n > 1) {
        n = (n + kScanChunk - 1) / kScanChunk;
        w += n;
    }
    return w + 1;
}

// Exclusive scan in place; ws holds scan_ws_words(n) words and must outlive the kernels
// (enqueued on s, no synchronisation here).
Status scan_exclusive(uint32_t *data, int64_t n, uint32_t *ws, hipStream_t s) {
    if (n <= 0) return Status::Ok();
    const int64_t nb = (n + kScanChunk - 1) / kScanChunk;
    hipLaunchKernelGGL(k_scan_block, dim3((unsigned)nb), dim3(kBlock), 0, s, data, n, ws);
    MWG_HIP(hipGetLastError());
    if (nb > 1) {
        MWG_TRY(scan_exclusive(ws, nb, ws + nb, s));
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kBlock), 0, s, data, n, ws);
        MWG_HIP(hipGetLastError());
    }
    return Status::Ok();
}

Status scan_exclusive(uint32_t *data, int64_t n, hipStream_t s) {
    Tmp ws;
    MWG_TRY(ws.alloc(4 * (size_t)scan_ws_words(n), s));
    MWG_TRY(scan_exclusive(data, n, ws.as<uint32_t>(), s));
    if (!ws.pooled()) MWG_HIP(hipStreamSynchronize(s));  // ws must outlive the kernels
    return Status::Ok();
}

// Sorts (keys, implicit index) by the low keybits bits; result in keys_out/vals_out. The
// histogram and scan scratch are allocated once for all passes; one synchronisation at
// the end.
Status radix_sort(uint32_t *keys, uint32_t *keys_alt, uint32_t *vals, uint32_t *vals_alt,
                  int64_t n, int keybits, uint32_t **keys_out, uint32_t **vals_out,
                  hipStream_t s, const uint32_t *vals_init = nullptr) {
    const int nblocks = (int)((n + kSortChunk - 1) / kSortChunk);
    const int64_t nh = (int64_t)256 * std::max(nblocks, 1);
    Tmp ws;
    MWG_TRY(ws.alloc(4 * (size_t)(nh + scan_ws_words(nh)), s));
    uint32_t *hist = ws.as<uint32_t>(), *sws = hist + nh;
    uint32_t *kin = keys, *kout = keys_alt, *vout = vals;
    const uint32_t *vin = vals_init;
    const int passes = (keybits + 7) / 8;
    if (passes == 0) return make_error(MW_ERR_UNSUPPORTED, "empty sort key");
    for (int p = 0; p < passes; p++) {
        const int shift = 8 * p;
        hipLaunchKernelGGL(k_rs_hist, dim3(nblocks), dim3(kBlock), 0, s, kin, n, shift, hist, nblocks);
        MWG_HIP(hipGetLastError());
        MWG_TRY(scan_exclusive(hist, nh, sws, s));
        hipLaunchKernelGGL(k_rs_scatter, dim3(nblocks), dim3(kBlock), 0, s, kin, vin, kout, vout,
                           hist, n, shift, nblocks);
        MWG_HIP(hipGetLastError());
        std::swap(kin, kout);
        vin = vout;
        vout = (vout == vals) ? vals_alt : vals;
    }
    *keys_out = kin;
    *vals_out = const_cast<uint32_t *>(vin); // after a pass vin is vals or vals_alt
    if (!ws.pooled()) MWG_HIP(hipStreamSynchronize(s));  // the scratch must outlive the kernels
    return Status::Ok();
}

__global__ void k_tile_bounds(const uint32_t *skeys, int64_t nkept, int cellbits, int32_t *tstart,
                              int32_t *tend) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nkept) return;
    const uint32_t t = skeys[i] >> cellbits;
    if (i == 0 || (skeys[i - 1] >> cellbits) != t) tstart[t] = (int32_t)i;
    if (i == nkept - 1 || (skeys[i + 1] >> cellbits) != t) tend[t] = (int32_t)(i + 1);
}

__global__ void k_gather(const uint32_t *perm, int64_t nkept, int nchan, const uint32_t *pos,
                         const float *weights, const uint32_t *ants, const int32_t *kidx,
                         uint32_t *spos, float *sw, uint32_t *sant, uint32_t *skid) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nkept) return;
    const uint32_t g = perm[i];
    spos[i] = pos[g];
    if (sw) sw[i] = weights[g];
    if (sant) sant[i] = ants[(int64_t)g / nchan];
    if (skid) skid[i] = (uint32_t)kidx[g];
}

// Per sorted group, the gridder's precomputed addressing: the footprint origin inside the
// haloed LDS tile (row stride STR) and the offsets of its two phase rows in the tap table
// with rows padded to 8 floats.
__global__ void k_codes(const uint32_t *spos, int64_t nkept, int tb, int STR, int W, int O,
                        uint32_t *code) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nkept) return;
    const uint32_t p = spos[i];
    const uint32_t mask = (1u << tb) - 1u;
    const uint32_t cx = p & 0xFFFu, cy = (p >> 12) & 0xFFFu;
    const uint32_t px = (p >> 24) & 0xFu, py = p >> 28;
    const uint32_t cell = (cy & mask) * (uint32_t)STR + (cx & mask);
    code[i] = cell | ((px * 8u) << 16) | ((py * 8u) << 24);
}

__global__ void k_pack_ants(const int32_t *a1, const int32_t *a2, int64_t nrow, uint32_t *out) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < nrow) out[r] = (uint32_t)a1[r] | ((uint32_t)a2[r] << 16);
}

// Counts entries of an index array outside [0, limit).
__global__ void k_count_out_of_range(const int32_t *idx, int64_t n, int32_t limit,
                                     unsigned long long *bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool out = i < n && (idx[i] < 0 || idx[i] >= limit);
    const unsigned long long m = __ballot(out);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(bad, (unsigned long long)__popcll(m));
}

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}


int bitlength(uint64_t v) {
    int r = 0;
    while (v) {
        r++;
        v >>= 1;
    }
    return r;
}

unsigned grid1d(int64_t n, int block = kBlock) { return (unsigned)((n + block - 1) / block); }

// Copy a caller array to the device (host source) or use it in place (device source).
template <class T>
Status stage_input(const T *src, size_t count, int mem, Tmp &tmp, const T **dst, hipStream_t s) {
    *dst = nullptr;
    if (!src) return Status::Ok();
    if (mem == MW_MEM_DEVICE) {
        *dst = src;
        return Status::Ok();
    }
    MWG_TRY(tmp.alloc(sizeof(T) * count, s));
    MWG_HIP(hipMemcpyAsync(tmp.p, src, sizeof(T) * count, hipMemcpyHostToDevice, s));
    *dst = (const T *)tmp.p;
    return Status::Ok();
}

} // namespace

// Library-internal entry points of the sort and scan (used by the kernel-stack schedule).
Status sort_pairs(uint32_t *keys, uint32_t *keys_alt, const uint32_t *vals_init, uint32_t *vals,
                  uint32_t *vals_alt, int64_t n, int keybits, uint32_t **keys_out,
                  uint32_t **vals_out, hipStream_t s) {
    return radix_sort(keys, keys_alt, vals, vals_alt, n, keybits, keys_out, vals_out, s, vals_init);
}

Status exclusive_scan_u32(uint32_t *data, int64_t n, hipStream_t s) { return scan_exclusive(data, n, s); }

Status launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s) {
    if (n <= 0) return Status::Ok();
    hipLaunchKernelGGL(k_fill_u32, dim3(grid1d(n)), dim3(kBlock), 0, s, p, n, v);
    MWG_HIP(hipGetLastError());
    return Status::Ok();
}

int tile_stride_host(int R, int W) {
    int st = R;
    while ((st - W) % 32 != 0) st++;
    return st;
}

// ------------------------------------------------------------------------------------------
// Work list: sort by (tile[, cell, row sub-position]), tile bounds, split heavy tiles,
// largest first.
// Rebuilt when the tuner changes the tile size, order or split.
// ------------------------------------------------------------------------------------------
Status rebuild_schedule(Instance &I, const Launch &L, hipStream_t s) {
    const int64_t ng = I.ngroups;
    const int tb = ilog2(L.tile);
    if ((1 << tb) != L.tile) return make_error(MW_ERR_INVALID_ARG, "tile %d is not a power of two", L.tile);
    const int ntx = (I.nx + L.tile - 1) / L.tile, nty = (I.ny + L.tile - 1) / L.tile;
    const int64_t ntiles = (int64_t)ntx * nty;
    const int cellbits = L.order != 2 ? 2 * tb + 4 : 0; // key bits below the tile index
    const uint64_t maxkey = (uint64_t)ntiles << cellbits; // exclusive bound of valid keys
    const int keybits = bitlength(maxkey);
    if (keybits > 31) return make_error(MW_ERR_UNSUPPORTED, "sort key wider than 31 bits");
    const uint32_t sentinel = (keybits >= 32) ? 0xFFFFFFFFu : ((1u << keybits) - 1u);

    const int64_t nk = I.nkept;
    const bool resort = !(L.tile == I.sorted_tile && L.order == I.sorted_order);
    if (resort) {
        Tmp keys, keys2, vals, vals2;
        MWG_TRY(keys.alloc(4 * ng, s));
        MWG_TRY(keys2.alloc(4 * ng, s));
        MWG_TRY(vals.alloc(4 * ng, s));
        MWG_TRY(vals2.alloc(4 * ng, s));
        uint32_t *skeys = nullptr, *sperm = nullptr;
        if (ng > 0) {
            // radial ranks from a per-cell table when there are more groups than cells
            Tmp ranks;
            const int64_t ncells = ntiles << (2 * tb);
            const bool table = L.order == 3 && tb <= 4 && ng > ncells;
            if (table) {
                MWG_TRY(ranks.alloc((size_t)ncells, s));
                hipLaunchKernelGGL(k_rank_table, dim3(grid1d(ncells)), dim3(kBlock), 0, s, tb, ntx, ncells, I.nx,
                                   I.ny, ranks.as<uint8_t>());
                MWG_HIP(hipGetLastError());
            }
            hipLaunchKernelGGL(k_keys, dim3(grid1d(ng)), dim3(kBlock), 0, s, I.pos, ng, tb, ntx, I.nx, I.ny, L.order,
                               sentinel, table ? ranks.as<uint8_t>() : (const uint8_t *)nullptr, keys.as<uint32_t>());
            MWG_HIP(hipGetLastError());
            MWG_TRY(radix_sort(keys.as<uint32_t>(), keys2.as<uint32_t>(), vals.as<uint32_t>(),
                               vals2.as<uint32_t>(), ng, keybits, &skeys, &sperm, s));
            MWG_HIP(hipMemcpyAsync(I.perm, sperm, 4 * ng, hipMemcpyDeviceToDevice, s));
        }
        // tile bounds
        Tmp tstart, tend;
        MWG_TRY(tstart.alloc(4 * ntiles, s));
        MWG_TRY(tend.alloc(4 * ntiles, s));
        MWG_TRY(launch_fill_u32(tstart.as<uint32_t>(), ntiles, 0, s));
        MWG_TRY(launch_fill_u32(tend.as<uint32_t>(), ntiles, 0, s));
        if (nk > 0) {
            hipLaunchKernelGGL(k_tile_bounds, dim3(grid1d(nk)), dim3(kBlock), 0, s, skeys, nk,
                               cellbits, tstart.as<int32_t>(), tend.as<int32_t>());
            MWG_HIP(hipGetLastError());
        }
        I.h_tstart.assign(ntiles, 0);
        I.h_tend.assign(ntiles, 0);
        MWG_HIP(hipMemcpyAsync(I.h_tstart.data(), tstart.p, 4 * ntiles, hipMemcpyDeviceToHost, s));
        MWG_HIP(hipMemcpyAsync(I.h_tend.data(), tend.p, 4 * ntiles, hipMemcpyDeviceToHost, s));
        MWG_HIP(hipStreamSynchronize(s));
        I.sorted_tile = L.tile;
        I.sorted_order = L.order;
    }
    const std::vector<int32_t> &hs = I.h_tstart, &he = I.h_tend;

    std::vector<WorkItem> items;
    int nonempty = 0;
    for (int64_t t = 0; t < ntiles; t++) {
        const int32_t b = hs[t], cnt = he[t] - hs[t];
        if (cnt <= 0) continue;
        nonempty++;
        if (cnt <= L.split) {
            items.push_back({(int32_t)t, b, b + cnt, 0});
            continue;
        }
        const int64_t pieces = (cnt + L.split - 1) / L.split;
        for (int64_t q = 0; q < pieces; q++)
            items.push_back({(int32_t)t, (int32_t)(b + cnt * q / pieces), (int32_t)(b + cnt * (q + 1) / pieces), 0});
    }
    if (L.schedule == 2) {
        // Z-order of tile coordinates (the split pieces of a tile stay together), so that
        // consecutive work items cover neighbouring tiles and share cached lines.
        auto morton = [ntx](int32_t t) {
            uint32_t x = (uint32_t)(t % ntx), y = (uint32_t)(t / ntx), m = 0;
            for (int b = 0; b < 16; b++) m |= ((x >> b) & 1u) << (2 * b) | ((y >> b) & 1u) << (2 * b + 1);
            return m;
        };
        std::stable_sort(items.begin(), items.end(), [&](const WorkItem &a, const WorkItem &b) {
            return morton(a.tile) < morton(b.tile);
        });
    } else {
        // largest first, ties in tile order: a stable counting sort on the item size
        int maxsz = 0;
        for (const WorkItem &w : items) maxsz = std::max(maxsz, w.end - w.begin);
        std::vector<int32_t> at((size_t)maxsz + 2, 0);
        for (const WorkItem &w : items) at[maxsz - (w.end - w.begin) + 1]++;
        for (int k = 0; k <= maxsz; k++) at[k + 1] += at[k];
        std::vector<WorkItem> sorted(items.size());
        for (const WorkItem &w : items) sorted[at[maxsz - (w.end - w.begin)]++] = w;
        items.swap(sorted);
    }
    // Schedule 2: the launch's workgroups are dealt to the 8 XCDs round-robin by index; the
    // logical workgroups (wg_waves consecutive work items each) are cut into 8 contiguous
    // chunks of about equal total groups, chunk x served by the workgroups of XCD x.
    {
        const int nw = L.wg_waves;
        const int nlog = (int)((items.size() + nw - 1) / nw);
        std::vector<int64_t> wsum(nlog + 1, 0);
        for (int b = 0; b < nlog; b++) {
            int64_t s_ = 0;
            for (int k = b * nw; k < std::min<int>((int)items.size(), (b + 1) * nw); k++)
                s_ += items[k].end - items[k].begin;
            wsum[b + 1] = wsum[b] + s_;
        }
        I.xcd_start[0] = 0;
        int maxlen = 0;
        for (int x = 1; x <= 8; x++) {
            const int64_t target = wsum[nlog] * x / 8;
            int b = I.xcd_start[x - 1];
            while (b < nlog && wsum[b] < target) b++;
            I.xcd_start[x] = (x == 8) ? nlog : b;
            maxlen = std::max(maxlen, I.xcd_start[x] - I.xcd_start[x - 1]);
        }
        I.xcd_wgs = maxlen;
    }
    // Schedule 3: an item of n groups is shared by nsub = 2^k >= n / (split / wg_waves)
    // (at most wg_waves) consecutive waves of one workgroup, wave j taking the j-th of nsub
    // equal parts. Items are in largest-first order, so nsub never grows along the list and
    // the items pack the workgroups' wave slots without gaps (only the last one is padded).
    std::vector<int2> &coop = I.h_coop;
    coop.clear();
    if (L.schedule == 3) {
        const int nw = L.wg_waves;
        const int64_t per = std::max(64, L.split / nw);
        for (size_t i = 0; i < items.size(); i++) {
            const int64_t n = items[i].end - items[i].begin;
            int nsub = 1;
            while (nsub < nw && (int64_t)nsub * per < n) nsub *= 2;
            if (coop.size() % nw + nsub > (size_t)nw) coop.resize((coop.size() / nw + 1) * nw, make_int2(-1, 0));
            for (int k = 0; k < nsub; k++) coop.push_back(make_int2((int)i, k | nsub << 8));
        }
        if (coop.size() % nw) coop.resize((coop.size() / nw + 1) * nw, make_int2(-1, 0));
    }
    // CSR of work items per tile (for the deterministic merge flush)
    std::vector<int32_t> &tw = I.h_tw, &ids = I.h_ids;
    tw.assign((size_t)ntiles + 1, 0);
    ids.assign(items.size(), 0);
    for (const WorkItem &w : items) tw[w.tile + 1]++;
    for (int64_t t = 0; t < ntiles; t++) tw[t + 1] += tw[t];
    {
        std::vector<int32_t> fillp(tw.begin(), tw.end() - 1);
        for (size_t i = 0; i < items.size(); i++) ids[fillp[items[i].tile]++] = (int32_t)i;
    }
    // Merge blocks that some work item's haloed tile reaches, then those none reaches.
    std::vector<int32_t> &mlist = I.h_mblocks;
    mlist.clear();
    int nmerge = 0;
    {
        // a block is reached when it meets the haloed extent [tx T - h, tx T + T - 1 + h] of
        // a tile with work items (per axis; blocks listed in row-major order)
        const int bpr = (I.nx + kMergeB - 1) / kMergeB, bpc = (I.ny + kMergeB - 1) / kMergeB;
        const int h = (I.W - 1) / 2, T = L.tile;
        std::vector<uint8_t> reach((size_t)bpr * bpc, 0);
        for (int64_t t = 0; t < ntiles; t++) {
            if (tw[t + 1] == tw[t]) continue;
            const int tx = (int)(t % ntx), ty = (int)(t / ntx);
            const int bx0 = std::max(0, tx * T - h) / kMergeB, bx1 = std::min(bpr - 1, (tx * T + T - 1 + h) / kMergeB);
            const int by0 = std::max(0, ty * T - h) / kMergeB, by1 = std::min(bpc - 1, (ty * T + T - 1 + h) / kMergeB);
            for (int by = by0; by <= by1; by++)
                for (int bx = bx0; bx <= bx1; bx++) reach[(size_t)by * bpr + bx] = 1;
        }
        mlist.reserve((size_t)bpr * bpc);
        for (int b = 0; b < bpr * bpc; b++)
            if (reach[b]) mlist.push_back(b);
        nmerge = (int)mlist.size();
        for (int b = 0; b < bpr * bpc; b++)
            if (!reach[b]) mlist.push_back(b);
    }
    // (re)allocate schedule arrays: these are small; keep them in the arena. The host lists
    // stay in the instance (the batched plan reads them, and the uploads are not waited for).
    I.h_work.swap(items);
    const std::vector<WorkItem> &work_list = I.h_work;
    I.L = L;
    I.ntx = ntx;
    I.nty = nty;
    I.ntiles_nonempty = nonempty;
    I.nwork = (int)work_list.size();
    I.max_work_groups = 0;
    for (const WorkItem &w : work_list) I.max_work_groups = std::max(I.max_work_groups, w.end - w.begin);
    void *p;
    if (I.cap_work < std::max<size_t>(work_list.size(), 1)) {
        I.cap_work = std::max<size_t>(work_list.size(), 1);
        MWG_TRY(I.arena.alloc(&p, sizeof(WorkItem) * I.cap_work));
        I.work = (WorkItem *)p;
        MWG_TRY(I.arena.alloc(&p, 4 * I.cap_work));
        I.work_ids = (int32_t *)p;
    }
    if (I.cap_tiles < (size_t)ntiles + 1) {
        I.cap_tiles = (size_t)ntiles + 1;
        MWG_TRY(I.arena.alloc(&p, 4 * I.cap_tiles));
        I.tile_work = (int32_t *)p;
    }
    if (!work_list.empty())
        MWG_HIP(hipMemcpyAsync(I.work, work_list.data(), sizeof(WorkItem) * work_list.size(),
                               hipMemcpyHostToDevice, s));
    I.coop_wgs = L.schedule == 3 ? (int)(coop.size() / L.wg_waves) : 0;
    if (!coop.empty()) {
        if (I.cap_coop < coop.size()) {
            I.cap_coop = coop.size();
            MWG_TRY(I.arena.alloc(&p, sizeof(int2) * I.cap_coop));
            I.coop = (int2 *)p;
        }
        MWG_HIP(hipMemcpyAsync(I.coop, coop.data(), sizeof(int2) * coop.size(), hipMemcpyHostToDevice, s));
    }
    MWG_HIP(hipMemcpyAsync(I.tile_work, tw.data(), 4 * (ntiles + 1), hipMemcpyHostToDevice, s));
    if (!ids.empty())
        MWG_HIP(hipMemcpyAsync(I.work_ids, ids.data(), 4 * ids.size(), hipMemcpyHostToDevice, s));
    if (!I.mblocks) { // the block count depends only on the grid size
        MWG_TRY(I.arena.alloc(&p, 4 * std::max<size_t>(mlist.size(), 1)));
        I.mblocks = (int32_t *)p;
    }
    MWG_HIP(hipMemcpyAsync(I.mblocks, mlist.data(), 4 * mlist.size(), hipMemcpyHostToDevice, s));
    I.n_mblocks = nmerge;
    I.n_zblocks = (int)mlist.size() - nmerge;

    // Sorted per-group arrays follow the new permutation.
    if (nk > 0) {
        if (resort) {
            hipLaunchKernelGGL(k_gather, dim3(grid1d(nk)), dim3(kBlock), 0, s, I.perm, nk, I.nchan, I.pos,
                               I.w_orig, I.ant_orig, I.kidx_orig, I.spos, I.sw, I.sant, I.skid);
            MWG_HIP(hipGetLastError());
        }
        if (!I.stacks) {
            const int R = L.tile + I.W - 1;
            hipLaunchKernelGGL(k_codes, dim3(grid1d(nk)), dim3(kBlock), 0, s, I.spos, nk, tb,
                               (L.variant == 4 || L.variant == 6) ? R : tile_stride_host(R, I.W), I.W, I.O,
                               I.scode);
            MWG_HIP(hipGetLastError());
        }
    }
    if (L.flush == 3) {
        bool built = false;
        MWG_TRY(build_owner_schedule(I, 0, &built, s));
    }
    if (L.variant == 6) MWG_TRY(build_block_schedule(I, s));
    return Status::Ok();
}

Status schedule_instance(Instance &I, const Launch &L, hipStream_t s) {
    MWG_TRY(rebuild_schedule(I, L, s));
    if (I.stacks) MWG_TRY(build_stack_schedule(I, L, s));
    I.scheduled = true;
    return Status::Ok();
}

size_t taplanes_lds(int npol, int T, int W, int O, int waves);
size_t collanes_lds(int npol, int T, int W, int O, int waves);
size_t wavetiles_lds(int npol, int T, int W, int O, int waves);
size_t owner_lds(int npol, int T, int W, int O, int waves);
size_t blocktiles_lds(int npol, int T, int W, int O, int waves);
size_t scatter_lds(int npol, int T, int W, int O);

static Launch default_launch(const Instance &I) {
    Launch L;
    // Work-item size: about 4096 items per instance (enough to fill the chip's wave slots
    // with a short tail), between 256 and 8192 groups.
    L.split = 256;
    while (L.split < 8192 && (int64_t)L.split * 4096 < I.nkept) L.split *= 2;
    L.order = 3;
    if (I.stacks) {
        // gather by output tile, one private tile per wavefront. On the beam x w-plane
        // workload (one polarisation) 16 x 16 tiles with tiles of more than 1024 candidates
        // split took 1.75 ms, against 2.06 ms splitting at 4096, 2.15 ms at 512, 2.78 ms
        // with 8 x 8 tiles and 3.21 ms with 32 x 32: more, shorter work items in flight.
        L.tile = 16;
        L.variant = 5;
        L.wg_waves = 8;
        L.flush = 1;
        L.split = 1024;
    } else if (I.W >= 3 && I.W <= 7) {
        // private 8x8 tiles per wavefront, merge pass: no LDS float atomics, no global atomics
        L.tile = 8;
        L.variant = 4;
        L.wg_waves = 4;
        L.flush = 2;
    } else {
        L.tile = I.npol >= 2 ? 32 : 64;
        L.variant = (I.W * I.W <= 64) ? 1 : 3;
        L.wg_waves = 8;
        L.flush = 1;
    }
    return L;
}

// Default launch overridden by the caller's non-zero tuning fields, checked against the
// kernels' limits (LDS, lanes).
Status resolve_launch(const Instance &I, const mw_tuning *t, Launch *out) {
    Launch L = default_launch(I);
    if (t) {
        if (t->tile) L.tile = t->tile;
        if (t->split) L.split = t->split;
        if (t->wg_waves) L.wg_waves = t->wg_waves;
        if (t->order) L.order = t->order;
        if (t->variant) L.variant = t->variant;
        if (t->flush) L.flush = t->flush;
        if (t->schedule) L.schedule = t->schedule;
    }
    if (L.schedule == 2 && L.variant != 4)
        return make_error(MW_ERR_UNSUPPORTED, "schedule 2 is implemented for variant 4 only");
    if (L.schedule == 3 && (L.variant != 4 || L.flush != 2))
        return make_error(MW_ERR_UNSUPPORTED, "schedule 3 is implemented for variant 4 with flush 2 only");
    if (L.schedule < 1 || L.schedule > 3) return make_error(MW_ERR_INVALID_ARG, "schedule %d", L.schedule);
    if (L.flush == 3 && (I.stacks || L.variant != 4 || L.schedule != 1))
        return make_error(MW_ERR_UNSUPPORTED, "flush 3 is implemented for variant 4 with schedule 1 only");
    if (L.flush == 3 && L.tile < I.W - 1)
        return make_error(MW_ERR_UNSUPPORTED, "flush 3 needs tiles of at least W - 1 cells");
    if (L.wg_waves < 4 && (I.stacks || (L.variant != 4 && L.variant != 6)))
        return make_error(MW_ERR_UNSUPPORTED, "workgroups of %d waves are implemented for variants 4 and 6 only", L.wg_waves);
    if (I.stacks) {
        L.variant = 5;
        if (L.wg_waves > 8)
            return make_error(MW_ERR_UNSUPPORTED, "the stack gridder takes at most 8 waves per workgroup (%d)",
                              L.wg_waves);
        const size_t lds = stack_lds(I.npol, L.tile, L.wg_waves);
        if (lds > 160 * 1024)
            return make_error(MW_ERR_UNSUPPORTED, "stack tiles need %zu B of LDS (tile %d, npol %d, %d waves)",
                              lds, L.tile, I.npol, L.wg_waves);
        if (L.tile < 8) return make_error(MW_ERR_UNSUPPORTED, "stack tiles must be >= 8");
    }
    if (!I.stacks) {
        if ((L.variant == 2 || L.variant == 4 || L.variant == 6) && (I.W > 7 || I.W < 3))
            return make_error(MW_ERR_UNSUPPORTED, "variants 2, 4 and 6 need 3 <= W <= 7 (W = %d)", I.W);
        if (L.variant == 6 && (L.flush == 3 || L.schedule != 1))
            return make_error(MW_ERR_UNSUPPORTED, "variant 6 takes flush 1 or 2 and schedule 1");
        if (L.variant == 1 && I.W * I.W > 64)
            return make_error(MW_ERR_UNSUPPORTED, "variant 1 needs W*W <= 64 (W = %d)", I.W);
        auto lds_of = [&](const Launch &X) {
            return X.variant == 1   ? taplanes_lds(I.npol, X.tile, I.W, I.O, X.wg_waves)
                   : X.variant == 2 ? collanes_lds(I.npol, X.tile, I.W, I.O, X.wg_waves)
                   : X.variant == 4 ? (X.flush == 3 ? owner_lds(I.npol, X.tile, I.W, I.O, X.wg_waves)
                                                    : wavetiles_lds(I.npol, X.tile, I.W, I.O, X.wg_waves))
                   : X.variant == 6 ? blocktiles_lds(I.npol, X.tile, I.W, I.O, X.wg_waves)
                                    : scatter_lds(I.npol, X.tile, I.W, I.O);
        };
        // private wave tiles of a large tile size may not fit: without an explicit variant,
        // fall back to the shared-tile kernel of the same lane layout
        if (L.variant == 4 && L.flush != 3 && !(t && t->variant) && L.schedule == 1 && lds_of(L) > 160 * 1024)
            L.variant = 2;
        // owner tiles of a large tile size: fewer waves per workgroup unless the caller set them
        if (L.variant == 4 && L.flush == 3 && !(t && t->wg_waves))
            while (L.wg_waves > 1 && lds_of(L) > 160 * 1024) L.wg_waves /= 2;
        const size_t lds = lds_of(L);
        if (lds > 160 * 1024)
            return make_error(MW_ERR_UNSUPPORTED, "launch needs %zu B of LDS (tile %d, npol %d)", lds,
                              L.tile, I.npol);
    }
    *out = L;
    return Status::Ok();
}

Status build_instance(Instance &I, const mw_instance &d, const mw_tuning *tuning, hipStream_t s, bool schedule,
                      bool count_tiles) {
    I.nx = d.nx;
    I.ny = d.ny;
    I.du = d.du;
    I.dv = d.dv;
    I.nrow = d.nrow;
    I.nchan = d.nchan;
    I.npol = d.npol;
    I.ngroups = d.nrow * d.nchan;
    I.O = d.oversample;
    I.stacks = d.kernel_stack != nullptr;
    I.W = I.stacks ? 0 : d.support;
    I.h = I.stacks ? 0 : (d.support - 1) / 2;
    I.has_weights = d.weights != nullptr;
    I.has_ants = d.ant1 != nullptr;
    I.nant = I.has_ants ? d.nant : 0;
    const int64_t ng = I.ngroups;

    // stage inputs
    Tmp t_uvw, t_freq, t_flags, t_w, t_a1, t_a2, t_kidx, t_ksup;
    const double *uvw, *freq;
    const uint8_t *flags;
    const float *weights;
    const int32_t *a1, *a2, *kidx = nullptr, *ksup = nullptr;
    MWG_TRY(stage_input(d.uvw_m, 3 * (size_t)d.nrow, d.mem, t_uvw, &uvw, s));
    MWG_TRY(stage_input(d.freq_hz, (size_t)d.nchan, d.mem, t_freq, &freq, s));
    MWG_TRY(stage_input(d.flags, (size_t)ng, d.mem, t_flags, &flags, s));
    MWG_TRY(stage_input(d.weights, (size_t)ng, d.mem, t_w, &weights, s));
    MWG_TRY(stage_input(d.ant1, (size_t)d.nrow, d.mem, t_a1, &a1, s));
    MWG_TRY(stage_input(d.ant2, (size_t)d.nrow, d.mem, t_a2, &a2, s));
    void *p;
    // Index arrays must stay inside the arrays they index (counted on the device). Kernel
    // indices are checked before the positions pass reads through them; antenna indices
    // together with the positions counts (nothing reads through them before that).
    Tmp bad;
    MWG_TRY(bad.alloc(sizeof(unsigned long long), s));
    MWG_TRY(launch_fill_u32(bad.as<uint32_t>(), 2, 0, s));
    if (a1 && d.nrow > 0) {
        hipLaunchKernelGGL(k_count_out_of_range, dim3(grid1d(d.nrow)), dim3(kBlock), 0, s, a1, (int64_t)d.nrow,
                           d.nant, bad.as<unsigned long long>());
        hipLaunchKernelGGL(k_count_out_of_range, dim3(grid1d(d.nrow)), dim3(kBlock), 0, s, a2, (int64_t)d.nrow,
                           d.nant, bad.as<unsigned long long>());
        MWG_HIP(hipGetLastError());
    }
    if (I.stacks && ng > 0) {
        MWG_TRY(stage_input(d.kernel_index, (size_t)ng, d.mem, t_kidx, &kidx, s));
        hipLaunchKernelGGL(k_count_out_of_range, dim3(grid1d(ng)), dim3(kBlock), 0, s, kidx, ng, d.nkernel,
                           bad.as<unsigned long long>());
        MWG_HIP(hipGetLastError());
        unsigned long long hb = 0;
        MWG_HIP(hipMemcpyAsync(&hb, bad.p, sizeof hb, hipMemcpyDeviceToHost, s));
        MWG_HIP(hipStreamSynchronize(s));
        if (hb) return make_error(MW_ERR_INVALID_ARG, "%llu antenna or kernel indices out of range", hb);
    }
    if (I.stacks) {
        I.nkernel = d.nkernel;
        MWG_TRY(stage_input(d.kernel_support, (size_t)d.nkernel, d.mem, t_ksup, &ksup, s));
        MWG_TRY(I.arena.alloc(&p, 8 * (size_t)d.kernel_elems));
        I.kstack = (float2 *)p;
        MWG_HIP(hipMemcpyAsync(I.kstack, d.kernel_stack, 8 * (size_t)d.kernel_elems,
                               d.mem == MW_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, s));
        MWG_TRY(I.arena.alloc(&p, 8 * (size_t)d.nkernel));
        I.koff = (int64_t *)p;
        MWG_HIP(hipMemcpyAsync(I.koff, d.kernel_offset, 8 * (size_t)d.nkernel,
                               d.mem == MW_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, s));
        MWG_TRY(I.arena.alloc(&p, 4 * (size_t)d.nkernel));
        I.ksup = (int32_t *)p;
        MWG_HIP(hipMemcpyAsync(I.ksup, d.kernel_support, 4 * (size_t)d.nkernel,
                               d.mem == MW_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, s));
        std::vector<int32_t> hsup(d.nkernel);
        std::vector<int64_t> hoff(d.nkernel);
        MWG_HIP(hipMemcpyAsync(hsup.data(), I.ksup, 4 * (size_t)d.nkernel, hipMemcpyDeviceToHost, s));
        MWG_HIP(hipMemcpyAsync(hoff.data(), I.koff, 8 * (size_t)d.nkernel, hipMemcpyDeviceToHost, s));
        MWG_HIP(hipStreamSynchronize(s));
        I.max_support = 0;
        for (int k = 0; k < d.nkernel; k++) {
            const int v = hsup[k];
            if (v < 1 || v > 63 || v % 2 == 0)
                return make_error(MW_ERR_INVALID_ARG, "kernel support %d must be odd in [1, 63]", v);
            const int64_t need = (int64_t)I.O * I.O * v * v;
            if (hoff[k] < 0 || hoff[k] + need > d.kernel_elems)
                return make_error(MW_ERR_INVALID_ARG, "kernel %d lies outside kernel_stack", k);
            I.max_support = std::max(I.max_support, v);
        }
    }

    // A1: positions
    MWG_TRY(I.arena.alloc(&p, 4 * (size_t)ng));
    I.pos = (uint32_t *)p;
    const int64_t pos_blocks = std::max<int64_t>(1, (int64_t)grid1d(ng));
    Tmp counts;
    MWG_TRY(counts.alloc(3 * sizeof(unsigned long long) + 12 * (size_t)pos_blocks, s));
    MWG_TRY(launch_fill_u32(counts.as<uint32_t>(), 6 + 3 * pos_blocks, 0, s));
    PosArgs a;
    a.ngroups = ng;
    a.nchan = I.nchan;
    a.nx = I.nx;
    a.ny = I.ny;
    a.O = I.O;
    a.h = I.h;
    a.du = I.du;
    a.dv = I.dv;
    a.uvw = uvw;
    a.freq = freq;
    a.flags = flags;
    a.weights = weights;
    a.kidx = kidx;
    a.ksup = ksup;
    a.pos = I.pos;
    a.blk_counts = counts.as<uint32_t>() + 6;
    a.wsel = d.wlo < d.whi ? 1 : 0;
    a.wlo = d.wlo;
    a.whi = d.whi;
    I.wsel = a.wsel != 0;
    I.wlo = d.wlo;
    I.whi = d.whi;
    if (ng > 0) {
        hipLaunchKernelGGL(k_positions, dim3(grid1d(ng)), dim3(kBlock), 0, s, a);
        MWG_HIP(hipGetLastError());
        const unsigned sb = (unsigned)std::min<int64_t>(kSumBlocks, (pos_blocks + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(k_sum_counts, dim3(sb), dim3(kBlock), 0, s, a.blk_counts, pos_blocks,
                           counts.as<unsigned long long>());
        MWG_HIP(hipGetLastError());
    }
    unsigned long long hc[3] = {0, 0, 0}, h8 = 0;
    Tmp tiles8;
    if (count_tiles) {
        const int ntx8 = (I.nx + kCountTile - 1) / kCountTile, nty8 = (I.ny + kCountTile - 1) / kCountTile;
        const int64_t nwords = ((int64_t)ntx8 * nty8 + 31) / 32;
        MWG_TRY(tiles8.alloc(8 + 4 * (size_t)nwords, s));
        uint32_t *bits = tiles8.as<uint32_t>() + 2;
        MWG_TRY(launch_fill_u32(bits, nwords, 0, s));
        if (ng > 0) {
            hipLaunchKernelGGL(k_mark_tiles, dim3(grid1d(ng)), dim3(kBlock), 0, s, I.pos, ng, ntx8, bits);
            MWG_HIP(hipGetLastError());
        }
        hipLaunchKernelGGL(k_popcount, dim3(1), dim3(kBlock), 0, s, bits, nwords,
                           tiles8.as<unsigned long long>());
        MWG_HIP(hipGetLastError());
        MWG_HIP(hipMemcpyAsync(&h8, tiles8.p, sizeof h8, hipMemcpyDeviceToHost, s));
    }
    unsigned long long hbad = 0;
    MWG_HIP(hipMemcpyAsync(&hbad, bad.p, sizeof hbad, hipMemcpyDeviceToHost, s));
    MWG_HIP(hipMemcpyAsync(hc, counts.p, sizeof hc, hipMemcpyDeviceToHost, s));
    MWG_HIP(hipStreamSynchronize(s));
    if (hbad) return make_error(MW_ERR_INVALID_ARG, "%llu antenna or kernel indices out of range", hbad);
    I.nkept = (int64_t)hc[0];
    I.nflagged = (int64_t)hc[1];
    I.noutside = (int64_t)hc[2];
    I.ntiles8 = (int64_t)h8;

    // Input-order copies the schedule gathers from (weights, packed antenna pairs, kernels).
    if (I.has_weights) {
        MWG_TRY(I.arena.alloc(&p, 4 * (size_t)std::max<int64_t>(ng, 1)));
        I.w_orig = (float *)p;
        if (ng > 0) MWG_HIP(hipMemcpyAsync(I.w_orig, weights, 4 * ng, hipMemcpyDeviceToDevice, s));
    }
    if (d.weighting != 0) {
        // density weighting: the weights every later call uses
        if (!I.w_orig) {
            MWG_TRY(I.arena.alloc(&p, 4 * (size_t)std::max<int64_t>(ng, 1)));
            I.w_orig = (float *)p;
        }
        MWG_TRY(apply_density_weighting(I, d.weighting, d.robust, weights, I.w_orig, s));
        I.has_weights = true;
    }
    if (I.has_ants) {
        MWG_TRY(I.arena.alloc(&p, 4 * (size_t)std::max<int64_t>(I.nrow, 1)));
        I.ant_orig = (uint32_t *)p;
        if (I.nrow > 0) {
            hipLaunchKernelGGL(k_pack_ants, dim3(grid1d(I.nrow)), dim3(kBlock), 0, s, a1, a2, I.nrow,
                               I.ant_orig);
            MWG_HIP(hipGetLastError());
        }
    }
    if (I.stacks) {
        MWG_TRY(I.arena.alloc(&p, 4 * (size_t)std::max<int64_t>(ng, 1)));
        I.kidx_orig = (int32_t *)p;
        if (ng > 0) MWG_HIP(hipMemcpyAsync(I.kidx_orig, kidx, 4 * ng, hipMemcpyDeviceToDevice, s));
    }
    // A2: sort + schedule (perm holds all ngroups: kept first, then dropped in input order)
    MWG_TRY(I.arena.alloc(&p, 4 * (size_t)std::max<int64_t>(ng, 1)));
    I.perm = (uint32_t *)p;
    I.dropped = I.perm + I.nkept;
    const int64_t nk = I.nkept;
    MWG_TRY(I.arena.alloc(&p, 4 * ((size_t)nk + 64)));  // + 64: the gridder reads ahead
    I.spos = (uint32_t *)p;
    MWG_TRY(I.arena.alloc(&p, 4 * ((size_t)nk + 64)));
    I.scode = (uint32_t *)p;
    if (I.has_weights) {
        MWG_TRY(I.arena.alloc(&p, 4 * (size_t)std::max<int64_t>(nk, 1)));
        I.sw = (float *)p;
    }
    if (I.has_ants) {
        MWG_TRY(I.arena.alloc(&p, 4 * (size_t)std::max<int64_t>(nk, 1)));
        I.sant = (uint32_t *)p;
    }
    if (I.stacks) {
        MWG_TRY(I.arena.alloc(&p, 4 * (size_t)std::max<int64_t>(nk, 1)));
        I.skid = (uint32_t *)p;
    }
    Launch L;
    MWG_TRY(resolve_launch(I, tuning, &L));
    I.tile_fixed = tuning && tuning->tile != 0;
    I.flush_fixed = tuning && tuning->flush != 0;
    I.L = L;
    if (schedule) MWG_TRY(schedule_instance(I, L, s));

    // prediction and calibration state (uvw, frequencies, per-antenna row lists)
    MWG_TRY(build_calibration(I, uvw, freq, a1, a2, s));

    // A3: kernel tables (built-in kernel) and correction vectors
    if (!I.stacks) {
        prolate_tables(I.W, I.O, I.nx, I.ny, I.h_tab, I.h_corrx, I.h_corry);
        // (host copies stay in the instance: the uploads below are not waited for here)
        std::vector<float> &taps2d = I.h_taps2d;
        taps2d.assign((size_t)I.O * I.O * 64, 0.0f);
        if (I.W * I.W <= 64) {
            for (int py = 0; py < I.O; py++)
                for (int px = 0; px < I.O; px++)
                    for (int sy = 0; sy < I.W; sy++)
                        for (int tx = 0; tx < I.W; tx++)
                            taps2d[((size_t)py * I.O + px) * 64 + sy * I.W + tx] =
                                I.h_tab[(size_t)py * I.W + sy] * I.h_tab[(size_t)px * I.W + tx];
        }
        MWG_TRY(I.arena.alloc(&p, 4 * taps2d.size()));
        I.taps2d = (float *)p;
        MWG_HIP(hipMemcpyAsync(I.taps2d, taps2d.data(), 4 * taps2d.size(), hipMemcpyHostToDevice, s));
        std::vector<float> &tabpad = I.h_tabpad;
        tabpad = I.h_tab;
        tabpad.resize(I.h_tab.size() + 8, 0.0f);  // uniform 8-float row reads past the last row
        MWG_TRY(I.arena.alloc(&p, 4 * tabpad.size()));
        I.tab = (float *)p;
        MWG_HIP(hipMemcpyAsync(I.tab, tabpad.data(), 4 * tabpad.size(), hipMemcpyHostToDevice, s));
        std::vector<float> &tab8 = I.h_tab8;
        tab8.assign((size_t)I.O * 8, 0.0f);
        for (int r = 0; r < I.O; r++)
            for (int t = 0; t < I.W && t < 8; t++) tab8[(size_t)r * 8 + t] = I.h_tab[(size_t)r * I.W + t];
        MWG_TRY(I.arena.alloc(&p, 4 * tab8.size()));
        I.tab8 = (float *)p;
        MWG_HIP(hipMemcpyAsync(I.tab8, tab8.data(), 4 * tab8.size(), hipMemcpyHostToDevice, s));
        MWG_TRY(I.arena.alloc(&p, 4 * (size_t)I.nx));
        I.corrx = (float *)p;
        MWG_HIP(hipMemcpyAsync(I.corrx, I.h_corrx.data(), 4 * (size_t)I.nx, hipMemcpyHostToDevice, s));
        MWG_TRY(I.arena.alloc(&p, 4 * (size_t)I.ny));
        I.corry = (float *)p;
        MWG_HIP(hipMemcpyAsync(I.corry, I.h_corry.data(), 4 * (size_t)I.ny, hipMemcpyHostToDevice, s));
    }
    return Status::Ok();
}

} // namespace mwg
