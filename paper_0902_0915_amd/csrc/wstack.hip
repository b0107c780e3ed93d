// w-stacking: the images of the w-planes of a plan (one instance per plane, each gridding
// only the groups of its w-range) summed with the w-term phase of their plane, an imaging
// variant beside the paper's coplanar imaging step.
//
// out[p] = sum_k images_k[p] exp(+2 pi i w_k (n - 1)), with n = sqrt(1 - l^2 - m^2) at pixel
// p (l = (x - nx/2) / (nx du), m = (y - ny/2) / (ny dv)). The transform of the image step has
// sign +i, so the plane's w-term enters with the same sign as its u and v terms. The pass is
// elementwise and bound by HBM: per pixel and polarisation it reads one complex value of every
// plane and writes one. n - 1 and the phase are formed in FP64 (|w (n - 1)| reaches many turns
// for large w), reduced to a fraction of a turn, then turned into FP32 sine and cosine.
#include "internal.h"

#include <cmath>

namespace mwg {

namespace {

constexpr int kMaxPlanes = 64;

struct WstackArgs {
    const float2 *img[kMaxPlanes];
    double w[kMaxPlanes];
    int nplanes, nx, ny, npol, accumulate;
    double du, dv;
};

__global__ __launch_bounds__(256) void k_wstack(WstackArgs a, float2 *out) {
    const int x = (int)(blockIdx.x * blockDim.x + threadIdx.x), y = (int)blockIdx.y;
    if (x >= a.nx) return;
    const double l = (double)(x - a.nx / 2) / ((double)a.nx * a.du);
    const double m = (double)(y - a.ny / 2) / ((double)a.ny * a.dv);
    const double n1 = sqrt(fmax(0.0, 1.0 - l * l - m * m)) - 1.0;
    const int64_t plane = (int64_t)a.nx * a.ny, pix = (int64_t)y * a.nx + x;
    float sr[4] = {0.f, 0.f, 0.f, 0.f}, si[4] = {0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < a.nplanes; k++) {
        const double t = a.w[k] * n1;  // turns
        const double fr = t - rint(t);
        float er, ei;
        sincospif(2.0f * (float)fr, &ei, &er);
        const float2 *src = a.img[k];
#pragma unroll
        for (int p = 0; p < 4; p++) {
            if (p >= a.npol) break;
            const float2 v = src[(int64_t)p * plane + pix];
            sr[p] += v.x * er - v.y * ei;
            si[p] += v.x * ei + v.y * er;
        }
    }
#pragma unroll
    for (int p = 0; p < 4; p++) {
        if (p >= a.npol) break;
        const int64_t idx = (int64_t)p * plane + pix;
        float2 o = make_float2(sr[p], si[p]);
        if (a.accumulate) {
            const float2 q = out[idx];
            o.x += q.x;
            o.y += q.y;
        }
        out[idx] = o;
    }
}

} // namespace

Status launch_wstack_combine(Plan &P, const void *const *images, float2 *out, int accumulate, hipStream_t s) {
    const int n = (int)P.inst.size();
    if (n > kMaxPlanes) return make_error(MW_ERR_UNSUPPORTED, "at most %d w-planes per combine (%d)", kMaxPlanes, n);
    const Instance &I0 = *P.inst[0];
    WstackArgs a{};
    for (int k = 0; k < n; k++) {
        const Instance &I = *P.inst[k];
        if (!I.wsel) return make_error(MW_ERR_STATE, "instance %d has no w-range", k);
        if (I.nx != I0.nx || I.ny != I0.ny || I.npol != I0.npol || I.du != I0.du || I.dv != I0.dv)
            return make_error(MW_ERR_STATE, "the w-planes must share grid size, cell size and polarisations");
        a.img[k] = (const float2 *)images[k];
        a.w[k] = 0.5 * (I.wlo + I.whi);
    }
    a.nplanes = n;
    a.nx = I0.nx;
    a.ny = I0.ny;
    a.npol = I0.npol;
    a.accumulate = accumulate;
    a.du = I0.du;
    a.dv = I0.dv;
    hipLaunchKernelGGL(k_wstack, dim3((unsigned)((I0.nx + 255) / 256), (unsigned)I0.ny), dim3(256), 0, s, a, out);
    MWG_HIP(hipGetLastError());
    return Status::Ok();
}

} // namespace mwg
