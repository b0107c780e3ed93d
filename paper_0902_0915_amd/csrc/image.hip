// Imaging: the FFT of the grid to one image per polarisation (Section 2: imaging "via a
// Fourier transform"; Table 1 "FFT") and the convolution correction (Table 1).
//
// direction +1: out[p] = sum_g in[g] exp(+2 pi i (g - n/2)(p - n/2)/n) in x and y, then
//               optionally out /= Cn(x) Cn(y).
// direction -1: the exact adjoint: optional division by Cn first, then the same transform
//               with sign -i.
// Centring uses the identity exp(2 pi i (g - n/2)(p - n/2)/n) =
// (-1)^g (-1)^p (-1)^(n/2) exp(2 pi i g p/n): a checkerboard sign before and after an
// ordinary unnormalised FFT, with the constant (-1)^((nx + ny)/2). Power-of-two grids use
// the library's own two-pass transform (fft.hip), which folds the signs and the correction
// into its loads and stores. Other sizes use rocFFT's single-precision in-place complex
// transform, batched over polarisations, between two scaling passes.
#include "internal.h"

#include <rocfft/rocfft.h>

#include <mutex>

namespace mwg {

namespace {

struct FftPlans {
    rocfft_plan fwd = nullptr, bwd = nullptr; // fwd = sign -i, bwd = sign +i
    rocfft_execution_info info = nullptr;
    void *work = nullptr;
    size_t work_bytes = 0;
};

std::once_flag g_rocfft_once;
rocfft_status g_rocfft_setup = rocfft_status_success;

// out = in * sign * (checker ? (-1)^(x+y) : 1) / (divide ? corrx[x] corry[y] : 1)
__global__ void k_image_scale(const float2 *in, float2 *out, int nx, int ny, int npol,
                              const float *corrx, const float *corry, int checker, int divide,
                              float sign) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    const int p = blockIdx.z;
    if (x >= nx || p >= npol) return;
    float f = sign;
    if (checker && ((x + y) & 1)) f = -f;
    const int64_t idx = ((int64_t)p * ny + y) * nx + x;
    float2 v = in[idx];
    if (divide) {
        const float c = corrx[x] * corry[y];
        v.x = v.x / c;
        v.y = v.y / c;
    }
    out[idx] = make_float2(f * v.x, f * v.y);
}

} // namespace

Status launch_image_scale(const float2 *in, float2 *out, int nx, int ny, int npol, const float *corrx,
                          const float *corry, int checker, int divide, hipStream_t s) {
    dim3 blk(256), grd((nx + 255) / 256, ny, npol);
    hipLaunchKernelGGL(k_image_scale, grd, blk, 0, s, in, out, nx, ny, npol, corrx, corry, checker,
                       divide, 1.0f);
    MWG_HIP(hipGetLastError());
    return Status::Ok();
}

#define MWG_FFT(expr)                                                                         \
    do {                                                                                      \
        rocfft_status st_ = (expr);                                                           \
        if (st_ != rocfft_status_success)                                                     \
            return make_error(MW_ERR_HIP, "%s failed: rocfft status %d", #expr, (int)st_);    \
    } while (0)

Status image_prepare(Instance &I) {
    if (I.fft) return Status::Ok();
    std::call_once(g_rocfft_once, [] { g_rocfft_setup = rocfft_setup(); });
    if (g_rocfft_setup != rocfft_status_success)
        return make_error(MW_ERR_HIP, "rocfft_setup failed: %d", (int)g_rocfft_setup);
    FftPlans *f = new FftPlans();
    I.fft = f;
    const size_t lengths[2] = {(size_t)I.nx, (size_t)I.ny}; // fastest dimension first
    MWG_FFT(rocfft_plan_create(&f->fwd, rocfft_placement_inplace, rocfft_transform_type_complex_forward,
                               rocfft_precision_single, 2, lengths, (size_t)I.npol, nullptr));
    MWG_FFT(rocfft_plan_create(&f->bwd, rocfft_placement_inplace, rocfft_transform_type_complex_inverse,
                               rocfft_precision_single, 2, lengths, (size_t)I.npol, nullptr));
    size_t w1 = 0, w2 = 0;
    MWG_FFT(rocfft_plan_get_work_buffer_size(f->fwd, &w1));
    MWG_FFT(rocfft_plan_get_work_buffer_size(f->bwd, &w2));
    f->work_bytes = std::max(w1, w2);
    MWG_FFT(rocfft_execution_info_create(&f->info));
    if (f->work_bytes) {
        MWG_TRY(I.arena.alloc(&f->work, f->work_bytes));
        MWG_FFT(rocfft_execution_info_set_work_buffer(f->info, f->work, f->work_bytes));
    }
    return Status::Ok();
}

void image_release(Instance &I) {
    FftPlans *f = (FftPlans *)I.fft;
    if (!f) return;
    if (f->fwd) rocfft_plan_destroy(f->fwd);
    if (f->bwd) rocfft_plan_destroy(f->bwd);
    if (f->info) rocfft_execution_info_destroy(f->info);
    delete f;
    I.fft = nullptr;
}

Status launch_image(Instance &I, const float2 *in, float2 *out, int direction, int correct,
                    hipStream_t s) {
    // the two-pass transform's column pass moves 16 bytes per lane: it needs a 16-byte aligned
    // output (a view at an odd complex offset goes through rocFFT instead)
    if (fft2d_supported(I.nx, I.ny) && ((uintptr_t)out & 15) == 0) {
        if (!I.twx) {
            MWG_TRY(fft2d_twiddles(I.arena, I.nx, &I.twx, s));
            MWG_TRY(fft2d_twiddles(I.arena, I.ny, &I.twy, s));
        }
        return launch_fft2d(in, out, I.nx, I.ny, I.npol, I.twx, I.twy, (const float *)I.corrx,
                            (const float *)I.corry, direction, correct, s);
    }
    MWG_TRY(image_prepare(I));
    FftPlans *f = (FftPlans *)I.fft;
    const float gsign = (((I.nx + I.ny) / 2) & 1) ? -1.0f : 1.0f;
    dim3 blk(256), grd((I.nx + 255) / 256, I.ny, I.npol);
    // pre: checkerboard (and the correction for the adjoint), in -> out
    hipLaunchKernelGGL(k_image_scale, grd, blk, 0, s, in, out, I.nx, I.ny, I.npol,
                       (const float *)I.corrx, (const float *)I.corry, 1,
                       (direction < 0 && correct) ? 1 : 0, 1.0f);
    MWG_HIP(hipGetLastError());
    MWG_FFT(rocfft_execution_info_set_stream(f->info, s));
    void *buf[1] = {out};
    MWG_FFT(rocfft_execute(direction > 0 ? f->bwd : f->fwd, buf, nullptr, f->info));
    // post: checkerboard, global sign (and the correction for the forward image), in place
    hipLaunchKernelGGL(k_image_scale, grd, blk, 0, s, (const float2 *)out, out, I.nx, I.ny, I.npol,
                       (const float *)I.corrx, (const float *)I.corry, 1,
                       (direction > 0 && correct) ? 1 : 0, gsign);
    MWG_HIP(hipGetLastError());
    return Status::Ok();
}

} // namespace mwg
