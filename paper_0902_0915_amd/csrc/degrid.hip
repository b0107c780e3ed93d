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
// loads). With four polarisations and supports 3, 5 and 7 the groups of one (cell, py) run
// share the contraction of the footprint's rows, formed once per run; otherwise each thread
// gathers one group's footprint. Per-antenna gradient sums accumulate in LDS and are added to HBM once per
// workgroup.
#include "internal.h"
#include "degrid_core.h"

#include <algorithm>

namespace mwg {

Status launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);

namespace {

template <int NPOL, int WT>
__global__ __launch_bounds__(1024) void k_degrid(DegridArgs a) {
    extern __shared__ __align__(16) float smem[];
    degrid_item<NPOL, WT>(a, a.work[blockIdx.x], smem);
}

// Four polarisations, supports 3, 5 and 7: groups of one (cell, py) run share their row
// contraction. (With one or two polarisations a group's own footprint read is short and the
// per-run bookkeeping costs more than it saves: the 96-job single-polarisation batch took
// 1.40 ms with the per-group form and 1.63 ms with runs.)
template <int NPOL, int W>
__global__ __launch_bounds__(256) void k_degrid_runs(DegridArgs a) {
    extern __shared__ __align__(16) float smem[];
    degrid_item_runs<NPOL, W>(a, a.work[blockIdx.x], smem);
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
    const int threads = degrid_threads(I.nkept, I.nwork);
    const dim3 grid((unsigned)I.nwork), block((unsigned)threads);
    a.ant_in_lds = 0;
    if (NPOL == 4 && (I.W == 3 || I.W == 5 || I.W == 7)) {
        size_t lds = degrid_runs_lds(NPOL, I.L.tile, I.W, I.O, threads / 64, 0);
        if (a.grad_gains && degrid_runs_lds(NPOL, I.L.tile, I.W, I.O, threads / 64, I.nant) <= 64 * 1024) {
            a.ant_in_lds = 1;
            lds = degrid_runs_lds(NPOL, I.L.tile, I.W, I.O, threads / 64, I.nant);
        }
        if (lds > 160 * 1024) return make_error(MW_ERR_UNSUPPORTED, "degrid tile needs %zu B of LDS", lds);
        switch (I.W) {
        case 3: hipLaunchKernelGGL((k_degrid_runs<NPOL, 3>), grid, block, lds, s, a); break;
        case 5: hipLaunchKernelGGL((k_degrid_runs<NPOL, 5>), grid, block, lds, s, a); break;
        default: hipLaunchKernelGGL((k_degrid_runs<NPOL, 7>), grid, block, lds, s, a); break;
        }
    } else {
        size_t lds = sizeof(float2) * (size_t)NPOL * R * R + 4 * (size_t)((I.O * I.W + 1) & ~1);
        if (a.grad_gains && lds + sizeof(float2) * (size_t)I.nant <= 64 * 1024) {
            a.ant_in_lds = 1;
            lds += sizeof(float2) * (size_t)I.nant;
        }
        if (lds > 160 * 1024) return make_error(MW_ERR_UNSUPPORTED, "degrid tile needs %zu B of LDS", lds);
        switch (I.W) {  // the common supports with their taps in registers
        case 3: hipLaunchKernelGGL((k_degrid<NPOL, 3>), grid, block, lds, s, a); break;
        case 5: hipLaunchKernelGGL((k_degrid<NPOL, 5>), grid, block, lds, s, a); break;
        case 7: hipLaunchKernelGGL((k_degrid<NPOL, 7>), grid, block, lds, s, a); break;
        default: hipLaunchKernelGGL((k_degrid<NPOL, 0>), grid, block, lds, s, a); break;
        }
    }
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
