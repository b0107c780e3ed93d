// Density weighting of a plan's visibilities (uniform and Briggs robust), an imaging variant
// beside the paper's gridding step (which grids with the data's own weights).
//
// The density of a grid cell is the summed weight W(c) of the kept groups centred in it.
// Uniform weighting divides each weight by its cell's density; robust weighting (Briggs 1995)
// by 1 + W(c) f^2 with f^2 = (5 * 10^-R)^2 / (sum_c W(c)^2 / sum_k w_k).
//
// The cell sums are formed with integer atomics on 64-bit fixed-point values (each weight
// rounded to a power-of-two grid chosen so that no cell sum can overflow): integer addition
// is associative, so the densities, and hence the weights and every grid built from them, do
// not depend on the order in which the GPU adds them.
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace mwg {

namespace {

constexpr int kBlock = 256;

unsigned grid1d(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

using Tmp = DevTmp;

__device__ inline int64_t cell_of(uint32_t p, int nx) {
    return (int64_t)((p >> 12) & 0xFFFu) * nx + (int64_t)(p & 0xFFFu);
}

// Largest |w| over kept groups, per block (as the bits of a non-negative float, so that an
// unsigned maximum orders them).
__global__ __launch_bounds__(kBlock) void k_wmax(const uint32_t *pos, const float *w, int64_t ng, uint32_t *out) {
    __shared__ uint32_t sm[kBlock];
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t v = 0;
    if (g < ng && pos[g] != kDropped) v = __float_as_uint(fabsf(w ? w[g] : 1.0f));
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int o = kBlock / 2; o >= 1; o >>= 1) {
        if ((int)threadIdx.x < o) sm[threadIdx.x] = max(sm[threadIdx.x], sm[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, sm[0]);
}

__global__ __launch_bounds__(kBlock) void k_density(const uint32_t *pos, const float *w, int64_t ng, int nx,
                                                     double scale, unsigned long long *cells) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ng) return;
    const uint32_t p = pos[g];
    if (p == kDropped) return;
    const long long q = llrint((double)(w ? w[g] : 1.0f) * scale);
    atomicAdd(cells + cell_of(p, nx), (unsigned long long)q);
}

// Per block: sum of W^2 and of W over cells (FP64), in a fixed tree order.
__global__ __launch_bounds__(kBlock) void k_density_sums(const unsigned long long *cells, int64_t n, double inv,
                                                          double2 *part) {
    __shared__ double a[kBlock], b[kBlock];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double x = i < n ? (double)(long long)cells[i] * inv : 0.0;
    a[threadIdx.x] = x * x;
    b[threadIdx.x] = x;
    __syncthreads();
    for (int o = kBlock / 2; o >= 1; o >>= 1) {
        if ((int)threadIdx.x < o) {
            a[threadIdx.x] += a[threadIdx.x + o];
            b[threadIdx.x] += b[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = make_double2(a[0], b[0]);
}

__global__ __launch_bounds__(kBlock) void k_density_total(const double2 *part, int64_t n, double2 *out) {
    __shared__ double a[kBlock], b[kBlock];
    double x = 0, y = 0;
    for (int64_t i = threadIdx.x; i < n; i += kBlock) {
        x += part[i].x;
        y += part[i].y;
    }
    a[threadIdx.x] = x;
    b[threadIdx.x] = y;
    __syncthreads();
    for (int o = kBlock / 2; o >= 1; o >>= 1) {
        if ((int)threadIdx.x < o) {
            a[threadIdx.x] += a[threadIdx.x + o];
            b[threadIdx.x] += b[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = make_double2(a[0], b[0]);
}

// w_out = w / W (mode 1) or w / (1 + W f2) (mode 2) for kept groups, 0 for dropped ones.
__global__ __launch_bounds__(kBlock) void k_density_apply(const uint32_t *pos, const float *w, int64_t ng, int nx,
                                                           const unsigned long long *cells, double inv, int mode,
                                                           const double2 *tot, double r5, float *out) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ng) return;
    const uint32_t p = pos[g];
    if (p == kDropped) {
        out[g] = 0.0f;
        return;
    }
    const double wg = w ? (double)w[g] : 1.0;
    const double W = (double)(long long)cells[cell_of(p, nx)] * inv;
    double r;
    if (mode == 1) {
        r = wg / W;
    } else {
        // f^2 = (5 10^-R)^2 / (sum W^2 / sum w); the total weight is the sum of the densities
        const double f2 = r5 * r5 / (tot->x / tot->y);
        r = wg / (1.0 + W * f2);
    }
    out[g] = (float)r;
}

} // namespace

Status apply_density_weighting(Instance &I, int mode, float robust, const float *w_in, float *w_out, hipStream_t s) {
    const int64_t ng = I.ngroups;
    if (ng == 0) return Status::Ok();
    Tmp mx;
    MWG_TRY(mx.alloc(4, s));
    MWG_HIP(hipMemsetAsync(mx.p, 0, 4, s));
    hipLaunchKernelGGL(k_wmax, dim3(grid1d(ng)), dim3(kBlock), 0, s, I.pos, w_in, ng, mx.as<uint32_t>());
    MWG_HIP(hipGetLastError());
    uint32_t hb = 0;
    MWG_HIP(hipMemcpyAsync(&hb, mx.p, 4, hipMemcpyDeviceToHost, s));
    MWG_HIP(hipStreamSynchronize(s));
    float wmax;
    std::memcpy(&wmax, &hb, 4);
    // fixed point: 2^e units per weight, with wmax * nkept * 2^e < 2^62 (no cell sum overflows)
    if (I.nkept == 0) {  // every group dropped: all weights 0 (the cell sums are never read)
        hipLaunchKernelGGL(k_density_apply, dim3(grid1d(ng)), dim3(kBlock), 0, s, I.pos, w_in, ng, I.nx,
                           (const unsigned long long *)nullptr, 1.0, 1, (const double2 *)nullptr, 0.0, w_out);
        MWG_HIP(hipGetLastError());
        MWG_HIP(hipStreamSynchronize(s));
        return Status::Ok();
    }
    const double bound = (double)wmax * (double)I.nkept;
    if (!(bound > 0.0) || !std::isfinite(bound))
        return make_error(MW_ERR_INVALID_ARG, "density weighting needs finite weights");
    const int e = std::min(60, (int)std::floor(62.0 - std::log2(bound)));
    const double scale = std::ldexp(1.0, e), inv = std::ldexp(1.0, -e);
    const int64_t ncell = (int64_t)I.nx * I.ny;
    Tmp cells;
    MWG_TRY(cells.alloc(8 * (size_t)ncell, s));
    MWG_HIP(hipMemsetAsync(cells.p, 0, 8 * (size_t)ncell, s));
    hipLaunchKernelGGL(k_density, dim3(grid1d(ng)), dim3(kBlock), 0, s, I.pos, w_in, ng, I.nx, scale,
                       cells.as<unsigned long long>());
    MWG_HIP(hipGetLastError());
    Tmp part, tot;
    const int64_t nb = grid1d(ncell);
    MWG_TRY(part.alloc(sizeof(double2) * (size_t)nb, s));
    MWG_TRY(tot.alloc(sizeof(double2), s));
    if (mode == 2) {
        hipLaunchKernelGGL(k_density_sums, dim3((unsigned)nb), dim3(kBlock), 0, s, cells.as<unsigned long long>(),
                           ncell, inv, part.as<double2>());
        hipLaunchKernelGGL(k_density_total, dim3(1), dim3(kBlock), 0, s, part.as<double2>(), nb, tot.as<double2>());
        MWG_HIP(hipGetLastError());
    }
    const double r5 = 5.0 * std::pow(10.0, -(double)robust);
    hipLaunchKernelGGL(k_density_apply, dim3(grid1d(ng)), dim3(kBlock), 0, s, I.pos, w_in, ng, I.nx,
                       cells.as<unsigned long long>(), inv, mode, tot.as<double2>(), r5, w_out);
    MWG_HIP(hipGetLastError());
    MWG_HIP(hipStreamSynchronize(s));
    return Status::Ok();
}

} // namespace mwg
