// Degridding: the exact adjoint of gridding, used as the backward pass of differentiable
// imaging. Each kept group gathers its W x W footprint of the grid with the same taps:
//   y[pol] = sum_{s,t} T[py][s] T[px][t] G[pol][cy+s][cx+t],
//   vis_out = w * conj(g1) * g2 * y,
// and, for the gradient with respect to the gains of the forward model w * g1 * conj(g2) * V,
//   grad_g[ant1] += g2 * conj(V) * (w y),   grad_g[ant2] += g1 * V * conj(w y).
// This is the gather form the paper's port used for its scatter loops (Section 3.2); here it
// is the transpose of the scatter rather than a replacement for it.
//
// One workgroup per work item stages the item's haloed tile of the grid in LDS (coalesced
// loads), then each thread gathers one group. Per-antenna gradient sums accumulate in LDS
// and are added to HBM once per workgroup.
#include "internal.h"

#include <algorithm>

namespace mwg {

Status launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);

namespace {

struct DegridArgs {
    const float2 *grid, *gains, *vis_in;
    float2 *vis_out, *grad_gains;
    const uint32_t *perm, *spos, *sant;
    const float *sw;
    const WorkItem *work;
    const float *tab;
    int nx, ny, T, ntx, W, O, nant, ant_in_lds;
};

template <int NPOL>
__global__ __launch_bounds__(1024) void k_degrid(DegridArgs a) {
    extern __shared__ __align__(16) float smem[];
    const int nthreads = blockDim.x, tid = threadIdx.x;
    const WorkItem wk = a.work[blockIdx.x];
    const int T = a.T, W = a.W, h = (W - 1) / 2, R = T + W - 1;
    const int tx0 = (wk.tile % a.ntx) * T, ty0 = (wk.tile / a.ntx) * T;
    float2 *g = (float2 *)smem;                      // [NPOL][R][R]
    float *tab = (float *)(g + (size_t)NPOL * R * R); // [O][W]
    float2 *gacc = (float2 *)(tab + ((a.O * W + 1) & ~1)); // [nant] when in LDS
    for (int idx = tid; idx < NPOL * R * R; idx += nthreads) {
        const int p = idx / (R * R), rc = idx - p * R * R;
        const int r = rc / R, c = rc - r * R;
        const int gy = ty0 - h + r, gx = tx0 - h + c;
        float2 v = make_float2(0.f, 0.f);
        if (gy >= 0 && gy < a.ny && gx >= 0 && gx < a.nx) v = a.grid[((int64_t)p * a.ny + gy) * a.nx + gx];
        g[idx] = v;
    }
    for (int i = tid; i < a.O * W; i += nthreads) tab[i] = a.tab[i];
    const bool want_g = a.grad_gains != nullptr;
    if (want_g && a.ant_in_lds)
        for (int i = tid; i < a.nant; i += nthreads) gacc[i] = make_float2(0.f, 0.f);
    __syncthreads();
    for (int64_t i = wk.begin + tid; i < wk.end; i += nthreads) {
        const uint32_t pp = a.spos[i];
        const int cx = (int)(pp & 0xFFFu), cy = (int)((pp >> 12) & 0xFFFu);
        const int px = (int)((pp >> 24) & 0xFu), py = (int)(pp >> 28);
        const int o = (cy - ty0) * R + (cx - tx0);
        float2 acc[NPOL];
#pragma unroll
        for (int p = 0; p < NPOL; p++) acc[p] = make_float2(0.f, 0.f);
        for (int sy = 0; sy < W; sy++) {
            const float ty = tab[py * W + sy];
            const float2 *row = g + o + sy * R;
            for (int sx = 0; sx < W; sx++) {
                const float tap = ty * tab[px * W + sx];
#pragma unroll
                for (int p = 0; p < NPOL; p++) {
                    const float2 v = row[(size_t)p * R * R + sx];
                    acc[p].x = fmaf(tap, v.x, acc[p].x);
                    acc[p].y = fmaf(tap, v.y, acc[p].y);
                }
            }
        }
        const float w = a.sw ? a.sw[i] : 1.0f;
#pragma unroll
        for (int p = 0; p < NPOL; p++) {
            acc[p].x *= w;
            acc[p].y *= w;
        }
        const uint32_t gi = a.perm[i];
        float2 out[NPOL];
        if (a.gains) {
            const uint32_t an = a.sant[i];
            const int a1 = (int)(an & 0xFFFFu), a2 = (int)(an >> 16);
            const float2 g1 = a.gains[a1], g2 = a.gains[a2];
            // conj(g1) * g2
            const float mr = g1.x * g2.x + g1.y * g2.y, mi = g1.x * g2.y - g1.y * g2.x;
#pragma unroll
            for (int p = 0; p < NPOL; p++)
                out[p] = make_float2(mr * acc[p].x - mi * acc[p].y, mr * acc[p].y + mi * acc[p].x);
            if (want_g) {
                float2 t1 = make_float2(0.f, 0.f), t2 = make_float2(0.f, 0.f);
                const float2 *vin = a.vis_in + (int64_t)gi * NPOL;
#pragma unroll
                for (int p = 0; p < NPOL; p++) {
                    const float2 V = vin[p], y = acc[p];
                    // conj(V) * y and V * conj(y)
                    const float cr = V.x * y.x + V.y * y.y, ci = V.x * y.y - V.y * y.x;
                    t1.x += cr;
                    t1.y += ci;
                    t2.x += cr;
                    t2.y -= ci;
                }
                // grad[a1] += g2 * t1 ; grad[a2] += g1 * t2
                const float2 d1 = make_float2(g2.x * t1.x - g2.y * t1.y, g2.x * t1.y + g2.y * t1.x);
                const float2 d2 = make_float2(g1.x * t2.x - g1.y * t2.y, g1.x * t2.y + g1.y * t2.x);
                float2 *dst = a.ant_in_lds ? gacc : a.grad_gains;
                atomicAdd(&dst[a1].x, d1.x);
                atomicAdd(&dst[a1].y, d1.y);
                atomicAdd(&dst[a2].x, d2.x);
                atomicAdd(&dst[a2].y, d2.y);
            }
        } else {
#pragma unroll
            for (int p = 0; p < NPOL; p++) out[p] = acc[p];
        }
        float2 *dst = a.vis_out + (int64_t)gi * NPOL;
#pragma unroll
        for (int p = 0; p < NPOL; p++) dst[p] = out[p];
    }
    if (want_g && a.ant_in_lds) {
        __syncthreads();
        for (int i = tid; i < a.nant; i += nthreads) {
            const float2 v = gacc[i];
            if (v.x != 0.0f) atomicAdd(&a.grad_gains[i].x, v.x);
            if (v.y != 0.0f) atomicAdd(&a.grad_gains[i].y, v.y);
        }
    }
}

template <int NPOL>
__global__ void k_zero_dropped(float2 *vis_out, const uint32_t *dropped, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float2 *dst = vis_out + (int64_t)dropped[i] * NPOL;
#pragma unroll
    for (int p = 0; p < NPOL; p++) dst[p] = make_float2(0.f, 0.f);
}

template <int NPOL>
Status launch_degrid_npol(Instance &I, DegridArgs &a, hipStream_t s) {
    const int ndropped = (int)(I.ngroups - I.nkept);
    if (ndropped > 0) {
        hipLaunchKernelGGL(k_zero_dropped<NPOL>, dim3((ndropped + 255) / 256), dim3(256), 0, s,
                           a.vis_out, (const uint32_t *)I.dropped, (int64_t)ndropped);
        MWG_HIP(hipGetLastError());
    }
    if (a.grad_gains) MWG_TRY(launch_fill_zero(a.grad_gains, sizeof(float2) * (size_t)I.nant, s));
    if (I.nwork == 0) return Status::Ok();
    const int R = I.L.tile + I.W - 1;
    size_t lds = sizeof(float2) * (size_t)NPOL * R * R + 4 * (size_t)((I.O * I.W + 1) & ~1);
    a.ant_in_lds = 0;
    if (a.grad_gains && lds + sizeof(float2) * (size_t)I.nant <= 64 * 1024) {
        a.ant_in_lds = 1;
        lds += sizeof(float2) * (size_t)I.nant;
    }
    if (lds > 160 * 1024) return make_error(MW_ERR_UNSUPPORTED, "degrid tile needs %zu B of LDS", lds);
    hipLaunchKernelGGL(k_degrid<NPOL>, dim3(I.nwork), dim3(256), lds, s, a);
    MWG_HIP(hipGetLastError());
    return Status::Ok();
}

} // namespace

Status launch_degrid(Instance &I, const float2 *grid, const float2 *gains, const float2 *vis_in,
                     float2 *vis_out, float2 *grad_gains, hipStream_t s) {
    if (I.stacks) return launch_degrid_stack(I, grid, gains, vis_in, vis_out, grad_gains, s);
    DegridArgs a{};
    a.grid = grid;
    a.gains = gains;
    a.vis_in = vis_in;
    a.vis_out = vis_out;
    a.grad_gains = grad_gains;
    a.perm = I.perm;
    a.spos = I.spos;
    a.sant = I.sant;
    a.sw = I.sw;
    a.work = I.work;
    a.tab = I.tab;
    a.nx = I.nx;
    a.ny = I.ny;
    a.T = I.L.tile;
    a.ntx = I.ntx;
    a.W = I.W;
    a.O = I.O;
    a.nant = I.nant;
    switch (I.npol) {
    case 1: return launch_degrid_npol<1>(I, a, s);
    case 2: return launch_degrid_npol<2>(I, a, s);
    case 4: return launch_degrid_npol<4>(I, a, s);
    default: return make_error(MW_ERR_UNSUPPORTED, "npol %d", I.npol);
    }
}

} // namespace mwg
