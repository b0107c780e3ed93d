// Stokes conversion of the four instrumental-polarisation images (Section 2.1: a 4 x 4
// matrix that depends on time and on the pixel's position relative to the instrument, applied
// at every pixel; Table 1 "Stokes Conversion").
//
// Input: the images of XX, XY, YX, YY as mw_image returns them, from visibilities gridded
// without their Hermitian mirror. Each mirrored sample (conj(V) at -uv, which for a cross
// polarisation is the mirror of the other cross product) would add the complex conjugate of
// an image, so the measured coherency matrix of a pixel is
//     E = [[2 Re XX, XY + conj(YX)], [YX + conj(XY), 2 Re YY]]   (Hermitian).
// With the instrument's response J toward the pixel (measured = J C J^H), the sky coherency is
// C = J^-1 E J^-H = adj(J) E adj(J)^H / |det J|^2, and for linear feeds
//     I = (C00 + C11)/2,  Q = (C00 - C11)/2,  U = Re C01,  V = Im C01.
// J = identity (no Jones field) reduces this to I = Re XX + Re YY, Q = Re XX - Re YY,
// U = Re XY + Re YX, V = Im XY - Im YX.
//
// The pass is elementwise and bound by HBM: per pixel it reads 32 B of images and 32 B of
// Jones matrix and writes 16 B. A thread takes two neighbouring pixels so that every access
// is a 16-byte load or an 8-byte store, coalesced along x.
#include "internal.h"

namespace mwg {

namespace {

struct C2 {
    float re, im;
};
__device__ inline C2 cm(C2 a, C2 b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline C2 cmc(C2 a, C2 b) { return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im}; } // a conj(b)
__device__ inline float abs2(C2 a) { return a.re * a.re + a.im * a.im; }

// Stokes (I, Q, U, V) of one pixel from its instrumental values and Jones matrix
// (j00, j01, j10, j11; has_j = 0: identity).
__device__ inline float4 pixel_stokes(C2 xx, C2 xy, C2 yx, C2 yy, const C2 (&j)[4], bool has_j) {
    const float a = 2.0f * xx.re, d = 2.0f * yy.re;
    const C2 b = {xy.re + yx.re, xy.im - yx.im};  // E01 = XY + conj(YX)
    if (!has_j) return make_float4(0.5f * (a + d), 0.5f * (a - d), b.re, b.im);
    // rows of adj(J): (j11, -j01) and (-j10, j00)
    const C2 r00 = j[3], r01 = {-j[1].re, -j[1].im}, r10 = {-j[2].re, -j[2].im}, r11 = j[0];
    const C2 det = {j[0].re * j[3].re - j[0].im * j[3].im - (j[1].re * j[2].re - j[1].im * j[2].im),
                    j[0].re * j[3].im + j[0].im * j[3].re - (j[1].re * j[2].im + j[1].im * j[2].re)};
    const float inv = 1.0f / abs2(det);
    // C_ik = sum_{l,m} A_il E_lm conj(A_km) with A = adj(J) and E = [[a, b], [conj b, d]]:
    // C_ii = a |A_i0|^2 + d |A_i1|^2 + 2 Re(A_i0 b conj(A_i1));
    // C_01 = a A00 conj(A10) + A00 b conj(A11) + A01 conj(b) conj(A10) + d A01 conj(A11).
    const float c00 = a * abs2(r00) + d * abs2(r01) + 2.0f * cmc(cm(r00, b), r01).re;
    const float c11 = a * abs2(r10) + d * abs2(r11) + 2.0f * cmc(cm(r10, b), r11).re;
    const C2 t1 = cmc(r00, r10), t2 = cmc(cm(r00, b), r11), t3 = cmc(r01, cm(r10, b)), t4 = cmc(r01, r11);
    const C2 c01 = {a * t1.re + t2.re + t3.re + d * t4.re, a * t1.im + t2.im + t3.im + d * t4.im};
    return make_float4(0.5f * (c00 + c11) * inv, 0.5f * (c00 - c11) * inv, c01.re * inv, c01.im * inv);
}

// One thread per pair of pixels (x, x + 1) of row y; npix2 = ny * nx / 2 pairs.
__global__ __launch_bounds__(256) void k_stokes(const float4 *__restrict__ img, const float4 *__restrict__ jones,
                                                float2 *__restrict__ out, int64_t npix2) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= npix2) return;
    float4 v[4];
#pragma unroll
    for (int p = 0; p < 4; p++) v[p] = img[(int64_t)p * npix2 + k];  // pixels 2k, 2k + 1 of plane p
    C2 j0[4], j1[4];
    const bool has_j = jones != nullptr;
    if (has_j) {
        const float4 a = jones[4 * k], b = jones[4 * k + 1], c = jones[4 * k + 2], e = jones[4 * k + 3];
        j0[0] = {a.x, a.y}; j0[1] = {a.z, a.w}; j0[2] = {b.x, b.y}; j0[3] = {b.z, b.w};
        j1[0] = {c.x, c.y}; j1[1] = {c.z, c.w}; j1[2] = {e.x, e.y}; j1[3] = {e.z, e.w};
    }
    const float4 s0 = pixel_stokes({v[0].x, v[0].y}, {v[1].x, v[1].y}, {v[2].x, v[2].y}, {v[3].x, v[3].y}, j0, has_j);
    const float4 s1 = pixel_stokes({v[0].z, v[0].w}, {v[1].z, v[1].w}, {v[2].z, v[2].w}, {v[3].z, v[3].w}, j1, has_j);
    out[k] = make_float2(s0.x, s1.x);
    out[npix2 + k] = make_float2(s0.y, s1.y);
    out[2 * npix2 + k] = make_float2(s0.z, s1.z);
    out[3 * npix2 + k] = make_float2(s0.w, s1.w);
}

} // namespace

Status launch_stokes(const Instance &I, const float2 *images, const float2 *jones, float *out, hipStream_t s) {
    if (I.npol != 4) return make_error(MW_ERR_STATE, "Stokes conversion needs an instance with 4 polarisations");
    if (((uintptr_t)images % 16) || ((uintptr_t)jones % 16) || ((uintptr_t)out % 8))
        return make_error(MW_ERR_INVALID_ARG, "images and jones must be 16-byte aligned, out 8-byte");
    const int64_t npix2 = (int64_t)I.nx * I.ny / 2;  // nx is even
    if (npix2 == 0) return Status::Ok();
    const int64_t nblk = (npix2 + 255) / 256;
    hipLaunchKernelGGL(k_stokes, dim3((unsigned)nblk), dim3(256), 0, s, (const float4 *)images,
                       (const float4 *)jones, (float2 *)out, npix2);
    MWG_HIP(hipGetLastError());
    return Status::Ok();
}

} // namespace mwg
