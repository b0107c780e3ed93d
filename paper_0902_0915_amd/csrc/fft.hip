// Two-pass image transform for power-of-two grids (64 ... 4096 on each axis): the centred,
// unnormalised 2-D FFT of the image step (Section 2, Table 1 "FFT") with the centring signs
// and the convolution correction (Table 1) folded into its loads and stores.
//
// Centring: exp(2 pi i s (g - n/2)(p - n/2)/n) = (-1)^g (-1)^p (-1)^(n/2) exp(2 pi i s g p/n)
// for even n, so the transform is an ordinary FFT with a checkerboard sign on the input and
// on the output and the constant (-1)^((nx + ny)/2).
//
// Pass 1 (rows): a workgroup loads whole rows (input sign, and for the adjoint the division
// by the correction, applied on the load), transforms them in LDS and writes them out.
// Pass 2 (columns): a workgroup loads C whole columns into LDS (~70 KB), transforms them and
// stores them with the output sign, the constant and, for the forward image, the division by
// the correction. Each pass reads and writes the image once.
//
// The 1-D transform is a Stockham self-sorting FFT with radix-8 passes (radix 4 or 2 for the
// last factor): butterfly i of a pass of span Ns reads elements i + r N/R, multiplies them
// by the twiddles exp(s 2 pi i r k / (Ns R)) with k = i mod Ns, takes an R-point DFT and
// writes the results to (i / Ns) Ns R + k + m Ns. The twiddle exp(s 2 pi i k / (Ns R)) comes
// from a table of exp(2 pi i j / N) computed in double precision; its powers r = 2 ... R - 1
// are formed by complex multiplication.
#include "internal.h"

#include <cmath>
#include <vector>

namespace mwg {

namespace {

constexpr float kRs2 = 0.70710678118654752440f;

__device__ inline float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ inline float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// s i z for s = +-1
__device__ inline float2 mul_si(float2 z, float s) { return make_float2(-s * z.y, s * z.x); }

// R-point DFT with sign s, natural order in and out: X[m] = sum_r x[r] exp(s 2 pi i r m / R).
__device__ inline void dft2(float2 &a, float2 &b) {
    const float2 t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

__device__ inline void dft4(float2 &x0, float2 &x1, float2 &x2, float2 &x3, float s) {
    const float2 a0 = cadd(x0, x2), a1 = csub(x0, x2), b0 = cadd(x1, x3), b1 = mul_si(csub(x1, x3), s);
    x0 = cadd(a0, b0);
    x2 = csub(a0, b0);
    x1 = cadd(a1, b1);
    x3 = csub(a1, b1);
}

template <int R>
__device__ inline void dft(float2 (&v)[R], float s) {
    if constexpr (R == 2) {
        dft2(v[0], v[1]);
    } else if constexpr (R == 4) {
        dft4(v[0], v[1], v[2], v[3], s);
    } else {
        // even and odd halves, then X[m] = E[m] + w^m O[m], X[m + 4] = E[m] - w^m O[m]
        dft4(v[0], v[2], v[4], v[6], s);
        dft4(v[1], v[3], v[5], v[7], s);
        const float2 t1 = cmul(v[3], make_float2(kRs2, s * kRs2));
        const float2 t2 = mul_si(v[5], s);
        const float2 t3 = cmul(v[7], make_float2(-kRs2, s * kRs2));
        const float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
        v[0] = cadd(e0, v[1]);
        v[4] = csub(e0, v[1]);
        v[1] = cadd(e1, t1);
        v[5] = csub(e1, t1);
        v[2] = cadd(e2, t2);
        v[6] = csub(e2, t2);
        v[3] = cadd(e3, t3);
        v[7] = csub(e3, t3);
    }
}

// LDS slot of element idx of a transform: one pad slot after every 16 elements, so that the
// stride-R writes of a Stockham pass fall in different banks.
__device__ inline int lpad(int idx) { return idx + (idx >> 4); }
template <int N>
constexpr int lds_len() { return N + N / 16; }

// One Stockham pass of radix R over a length-N sequence in LDS (buf, padded by lpad), T
// threads (thread lt) each taking NB = N / (R T) butterflies, with twiddles w1 = the table
// entries exp(2 pi i k / (Ns R)) of its butterflies. Reads everything before writing.
template <int N, int T, int R>
__device__ inline void stockham_pass(float2 *buf, int lt, int Ns, const float2 (&w1)[N / (R * T)], float s) {
    constexpr int NB = N / (R * T);
    float2 v[NB][R];
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int i = lt + b * T;
#pragma unroll
        for (int r = 0; r < R; r++) v[b][r] = buf[lpad(i + r * (N / R))];
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int i = lt + b * T;
        const int k = i & (Ns - 1);
        const float2 w = make_float2(w1[b].x, s * w1[b].y);
        float2 wr = w;
#pragma unroll
        for (int r = 1; r < R; r++) {
            v[b][r] = cmul(v[b][r], wr);
            if (r + 1 < R) wr = cmul(wr, w);
        }
        dft<R>(v[b], s);
        const int base = (i - k) * R + k;
#pragma unroll
        for (int m = 0; m < R; m++) buf[lpad(base + m * Ns)] = v[b][m];
    }
    __syncthreads();
}

constexpr int log2c(int n) { return n <= 1 ? 0 : 1 + log2c(n / 2); }

// The twiddles of every pass of a length-N transform for thread lt, loaded at once (so that
// their latency overlaps the data loads), and the passes themselves: radix 8, then one
// radix-4 or radix-2 pass for the remaining factor.
template <int N, int T>
struct FftTwiddles {
    static constexpr int P8 = log2c(N) / 3;
    static constexpr int RL = (log2c(N) % 3 == 2) ? 4 : ((log2c(N) % 3 == 1) ? 2 : 0);
    static constexpr int NB8 = N / (8 * T);
    static constexpr int NBL = RL ? N / (RL * T) : 1;
    float2 w8[P8][NB8];
    float2 wl[NBL];
    __device__ inline void load(int lt, const float2 *tw) {
        int Ns = 1;
#pragma unroll
        for (int p = 0; p < P8; p++, Ns *= 8) {
#pragma unroll
            for (int b = 0; b < NB8; b++) w8[p][b] = tw[((lt + b * T) & (Ns - 1)) * (N / (Ns * 8))];
        }
        if constexpr (RL != 0) {
#pragma unroll
            for (int b = 0; b < NBL; b++) wl[b] = tw[((lt + b * T) & (Ns - 1)) * (N / (Ns * RL))];
        }
    }
    __device__ inline void run(float2 *buf, int lt, float s) const {
        int Ns = 1;
#pragma unroll
        for (int p = 0; p < P8; p++, Ns *= 8) stockham_pass<N, T, 8>(buf, lt, Ns, w8[p], s);
        if constexpr (RL == 4) stockham_pass<N, T, 4>(buf, lt, Ns, wl, s);
        if constexpr (RL == 2) stockham_pass<N, T, 2>(buf, lt, Ns, wl, s);
    }
};

struct ScaleArgs {
    const float *corrx, *corry;
    float gsign;
    int divide_in, divide_out; // correction on the load (adjoint) / on the store (forward)
};

// Pass 1: rows. N = nx, T = N / 8 threads per row, B rows per workgroup.
template <int N, int T>
__global__ __launch_bounds__(512) void k_fft_rows(const float2 *in, float2 *out, int ny, int nrows,
                                                  const float2 *tw, float s, ScaleArgs sc) {
    extern __shared__ __align__(16) float2 lds[];
    const int B = blockDim.x / T;
    const int rb = threadIdx.x / T, lt = threadIdx.x % T;
    const int row = blockIdx.x * B + rb; // p * ny + y
    float2 *buf = lds + rb * lds_len<N>();
    const bool live = row < nrows;
    const int y = live ? row % ny : 0;
    const float cy = sc.divide_in ? sc.corry[y] : 1.0f;
    FftTwiddles<N, T> tws;
    tws.load(lt, tw);
    if (live) {
        const float2 *src = in + (int64_t)row * N;
#pragma unroll
        for (int e = 0; e < N / T; e++) {
            const int x = lt + e * T;
            float2 v = src[x];
            float f = ((x + y) & 1) ? -1.0f : 1.0f;
            if (sc.divide_in) f = f / (sc.corrx[x] * cy);
            buf[lpad(x)] = make_float2(f * v.x, f * v.y);
        }
    }
    __syncthreads();
    tws.run(buf, lt, s);
    if (live) {
        float2 *dst = out + (int64_t)row * N;
#pragma unroll
        for (int e = 0; e < N / T; e++) dst[lt + e * T] = buf[lpad(lt + e * T)];
    }
}

// Pass 2: columns, in place. N = ny, T = N / 16 threads per column, C columns per
// workgroup. Loads and stores go column-fastest, two columns (16 bytes) per lane; the
// transforms run with the threads of a wave on one column. The column stride in LDS is
// 2 mod 16 slots, so the column-fastest accesses hit different banks. Workgroups b, b + 8, ...
// (the same XCD when workgroups are dealt to the 8 XCDs in turn) take the neighbouring strips
// that share cache lines. The output must be 16-byte aligned.
template <int N, int T, int C>
__global__ __launch_bounds__(1024) void k_fft_cols(float2 *data, int nx, const float2 *tw, float s,
                                                   ScaleArgs sc) {
    extern __shared__ __align__(16) float2 lds[];
    constexpr int S = lds_len<N>() + 2;
    constexpr int H = C / 2;         // lanes per row
    constexpr int RP = (T * C) / H;  // rows per round
    const int nstrip = nx / C;
    // the L = 16 / C strips of one 128-byte line go to workgroups b, b + 8, ... (one XCD)
    constexpr int L = C >= 16 ? 1 : 16 / C;
    int b = blockIdx.x;
    if ((int)(gridDim.x / (8 * L)) * 8 * L > b) b = (b / (8 * L)) * 8 * L + (b % 8) * L + (b / 8) % L;
    const int p = b / nstrip, x0 = (b % nstrip) * C;
    const int tid = threadIdx.x, h = tid % H, r0 = tid / H;
    FftTwiddles<N, T> tws;
    tws.load(tid % T, tw);
    // global -> LDS
    {
        const float4 *src = (const float4 *)(data + (int64_t)p * N * nx + x0) + h;
#pragma unroll
        for (int y = r0; y < N; y += RP) {
            const float4 v = src[(int64_t)y * (nx / 2)];
            lds[(2 * h) * S + lpad(y)] = make_float2(v.x, v.y);
            lds[(2 * h + 1) * S + lpad(y)] = make_float2(v.z, v.w);
        }
    }
    __syncthreads();
    tws.run(lds + (tid / T) * S, tid % T, s);
    // LDS -> global with the output sign, the constant and the correction
    {
        float4 *dst = (float4 *)(data + (int64_t)p * N * nx + x0) + h;
        const int x = x0 + 2 * h;
        const float cx0 = sc.divide_out ? sc.corrx[x] : 1.0f, cx1 = sc.divide_out ? sc.corrx[x + 1] : 1.0f;
#pragma unroll
        for (int y = r0; y < N; y += RP) {
            float f0 = ((x + y) & 1) ? -sc.gsign : sc.gsign;
            float f1 = -f0;
            if (sc.divide_out) {
                const float cy = sc.corry[y];
                f0 = f0 / (cx0 * cy);
                f1 = f1 / (cx1 * cy);
            }
            const float2 v0 = lds[(2 * h) * S + lpad(y)], v1 = lds[(2 * h + 1) * S + lpad(y)];
            dst[(int64_t)y * (nx / 2)] = make_float4(f0 * v0.x, f0 * v0.y, f1 * v1.x, f1 * v1.y);
        }
    }
}

template <int N>
Status launch_rows(const float2 *in, float2 *out, int ny, int npol, const float2 *tw, float s,
                   const ScaleArgs &sc, hipStream_t st) {
    constexpr int T = N / 8;
    const int B = T >= 256 ? 1 : 256 / T;
    const int nrows = ny * npol;
    const size_t lds = sizeof(float2) * (size_t)B * lds_len<N>();
    hipLaunchKernelGGL((k_fft_rows<N, T>), dim3((nrows + B - 1) / B), dim3(B * T), lds, st, in, out, ny, nrows,
                       tw, s, sc);
    MWG_HIP(hipGetLastError());
    return Status::Ok();
}

template <int N>
Status launch_cols(float2 *data, int nx, int npol, const float2 *tw, float s, const ScaleArgs &sc,
                   hipStream_t st) {
    constexpr int T = N / 16;
    // columns per workgroup: about 70 KB of LDS, so that two workgroups share a CU
    constexpr int C = (8192 / N) > 16 ? 16 : 8192 / N;
    static_assert(C >= 2 && (C & 1) == 0, "two columns per lane");
    if (nx % C != 0) return make_error(MW_ERR_UNSUPPORTED, "nx %d not a multiple of %d", nx, C);
    const size_t lds = sizeof(float2) * (size_t)C * (lds_len<N>() + 2);
    hipLaunchKernelGGL((k_fft_cols<N, T, C>), dim3((nx / C) * npol), dim3(T * C), lds, st, data, nx, tw, s, sc);
    MWG_HIP(hipGetLastError());
    return Status::Ok();
}

bool pow2_in_range(int n) { return n >= 64 && n <= 4096 && (n & (n - 1)) == 0; }

} // namespace

bool fft2d_supported(int nx, int ny) { return pow2_in_range(nx) && pow2_in_range(ny); }

// Twiddle table exp(2 pi i j / n), j < n, as float2, built in double precision.
Status fft2d_twiddles(DevArena &arena, int n, float2 **out, hipStream_t s) {
    std::vector<float2> h(n);
    for (int j = 0; j < n; j++) {
        const double a = 2.0 * M_PI * (double)j / (double)n;
        h[j] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    void *p;
    MWG_TRY(arena.alloc(&p, sizeof(float2) * (size_t)n));
    MWG_HIP(hipMemcpyAsync(p, h.data(), sizeof(float2) * (size_t)n, hipMemcpyHostToDevice, s));
    MWG_HIP(hipStreamSynchronize(s));
    *out = (float2 *)p;
    return Status::Ok();
}

Status launch_fft2d(const float2 *in, float2 *out, int nx, int ny, int npol, const float2 *twx,
                    const float2 *twy, const float *corrx, const float *corry, int direction, int correct,
                    hipStream_t st) {
    const float s = direction > 0 ? 1.0f : -1.0f;
    ScaleArgs sc;
    sc.corrx = corrx;
    sc.corry = corry;
    sc.gsign = (((nx + ny) / 2) & 1) ? -1.0f : 1.0f;
    sc.divide_in = (direction < 0 && correct) ? 1 : 0;
    sc.divide_out = (direction > 0 && correct) ? 1 : 0;
    switch (nx) {
    case 64: MWG_TRY(launch_rows<64>(in, out, ny, npol, twx, s, sc, st)); break;
    case 128: MWG_TRY(launch_rows<128>(in, out, ny, npol, twx, s, sc, st)); break;
    case 256: MWG_TRY(launch_rows<256>(in, out, ny, npol, twx, s, sc, st)); break;
    case 512: MWG_TRY(launch_rows<512>(in, out, ny, npol, twx, s, sc, st)); break;
    case 1024: MWG_TRY(launch_rows<1024>(in, out, ny, npol, twx, s, sc, st)); break;
    case 2048: MWG_TRY(launch_rows<2048>(in, out, ny, npol, twx, s, sc, st)); break;
    case 4096: MWG_TRY(launch_rows<4096>(in, out, ny, npol, twx, s, sc, st)); break;
    default: return make_error(MW_ERR_UNSUPPORTED, "fft rows: nx %d", nx);
    }
    switch (ny) {
    case 64: return launch_cols<64>(out, nx, npol, twy, s, sc, st);
    case 128: return launch_cols<128>(out, nx, npol, twy, s, sc, st);
    case 256: return launch_cols<256>(out, nx, npol, twy, s, sc, st);
    case 512: return launch_cols<512>(out, nx, npol, twy, s, sc, st);
    case 1024: return launch_cols<1024>(out, nx, npol, twy, s, sc, st);
    case 2048: return launch_cols<2048>(out, nx, npol, twy, s, sc, st);
    case 4096: return launch_cols<4096>(out, nx, npol, twy, s, sc, st);
    default: return make_error(MW_ERR_UNSUPPORTED, "fft columns: ny %d", ny);
    }
}

} // namespace mwg
