// Calibration: the measurement loop over catalogue sources (Section 2: per-antenna complex
// gains from a linear least-squares fit to observed catalogue sources; Section 2.1: the
// contribution of catalogue sources is measured and removed in decreasing order of predicted
// flux, each measurement constraining the antenna gains; Table 1, "CML").
//
// Prediction. A point source (l, m, S) contributes S exp(-2 pi i (u l + v m + w (n - 1))) to a
// sample at (u, v, w) = uvw * f / c. The phase of a sample is large (thousands of turns at
// MWA baselines), so its path length and the product with f / c are formed in FP64 and
// reduced to a fraction of a turn before the FP32 sine and cosine.
//
// Gain solve. The data are modelled as V = g[a1] conj(g[a2]) M. The alternating least-squares
// iteration of Salvini & Wijnholds (2014, "StEFCal") solves, for every antenna p with the
// others fixed, g_p = sum w z conj(R) / sum w |z|^2 over all samples involving p (see the
// oracle for the derivation), damping every second iterate by averaging it with the previous
// one. With scalar gains constant over the data, every sample of one antenna pair has the same
// two gains, so the sums factor through two numbers per pair that do not depend on g:
//     P_b = sum_{rows of b, chan, pol} w conj(M) V,    Q_b = sum w |M|^2.
// Antenna p then needs num_p = sum_{a1(b) = p} g[a2] P_b + sum_{a2(b) = p} g[a1] conj(P_b) and
// den_p = sum_{a1 = p} |g[a2]|^2 Q_b + sum_{a2 = p} |g[a1]|^2 Q_b. One pass over the
// visibilities forms (P, Q) (the rows of a pair, one time step each, are found through a list
// built with the plan); every iteration after that reads only the pairs' (P, Q) through a
// per-antenna list of pairs, so the iterations cost almost nothing.
//
// Peeling. For each source in decreasing |S| (ties in catalogue order): (P, Q) of the current
// residual against the source's prediction, the iterations from unit gains, then the
// residual minus g[a1] conj(g[a2]) times the prediction. The subtraction of one source and
// the (P, Q) of the next share one pass over the residual (read once, written once).
// Everything is enqueued on the caller's stream; the only host work is ordering the catalogue.
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <unordered_map>
#include <vector>

namespace mwg {

namespace {

constexpr double kC = 299792458.0;
constexpr int kBlock = 256;

unsigned grid1d(int64_t n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

// exp(-2 pi i t) for t in turns (FP64), after reduction to [-1/2, 1/2] turn, by the hardware
// sine and cosine, whose input is in turns (over [-1/2, 1/2] turn their largest absolute
// error, measured against FP64, is 1.3e-7, the size of the rounding of the reduced phase to
// FP32; the library sincospif reaches 5e-8 at several times the instruction count)
__device__ inline float2 turn_phasor(double t) {
    const float fr = (float)(t - rint(t));
    return make_float2(__builtin_amdgcn_cosf(fr), -__builtin_amdgcn_sinf(fr));
}

struct Src {
    double l, m, n1, flux;  // n1 = sqrt(1 - l^2 - m^2) - 1
};

// Model visibilities of nsrc point sources (sources in global memory, read as uniform scalar
// loads), times g[a1] conj(g[a2]) when gains are given; written or added to out [ng][npol].
// Cross polarisations (1, 2 of 4) of an unpolarised source are zero. One thread per row and
// run of kPredChan consecutive channels: a source's path length u l + v m + w (n - 1) is
// formed once for the run, and only its product with each channel's f / c per channel.
constexpr int kPredChan = 4;

__global__ __launch_bounds__(kBlock) void k_predict(const double *uvw, const double *kf, int64_t nrow, int nchan,
                                                    int npol, const Src *src, int nsrc, const float2 *gains,
                                                    const uint32_t *ants, float2 *out, int accumulate) {
    const int nrun = (nchan + kPredChan - 1) / kPredChan;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nrow * nrun) return;
    const int64_t r = t / nrun;
    const int c0 = (int)(t - r * nrun) * kPredChan;
    const int nc = min(kPredChan, nchan - c0);
    double k[kPredChan];
#pragma unroll
    for (int q = 0; q < kPredChan; q++) k[q] = kf[c0 + (q < nc ? q : 0)];
    const double u = uvw[3 * r], v = uvw[3 * r + 1], w = uvw[3 * r + 2];
    float sr[kPredChan], si[kPredChan];
#pragma unroll
    for (int q = 0; q < kPredChan; q++) sr[q] = si[q] = 0.f;
    for (int j = 0; j < nsrc; j++) {
        const Src s = src[j];
        const double path = u * s.l + v * s.m + w * s.n1;
        const float flux = (float)s.flux;
#pragma unroll
        for (int q = 0; q < kPredChan; q++) {
            const float2 e = turn_phasor(path * k[q]);
            sr[q] += flux * e.x;
            si[q] += flux * e.y;
        }
    }
    float gr = 1.f, gi = 0.f;  // g1 conj(g2)
    if (gains) {
        const uint32_t an = ants[r];
        const float2 g1 = gains[an & 0xFFFFu], g2 = gains[an >> 16];
        gr = g1.x * g2.x + g1.y * g2.y;
        gi = g1.y * g2.x - g1.x * g2.y;
    }
#pragma unroll
    for (int q = 0; q < kPredChan; q++) {
        if (q >= nc) break;
        float mr = sr[q], mi = si[q];
        if (gains) {
            const float tr = gr * mr - gi * mi, ti = gr * mi + gi * mr;
            mr = tr;
            mi = ti;
        }
        float2 *o = out + (r * nchan + c0 + q) * npol;
        for (int p = 0; p < npol; p++) {
            const bool cross = npol == 4 && (p == 1 || p == 2);
            float2 val = cross ? make_float2(0.f, 0.f) : make_float2(mr, mi);
            if (accumulate) {
                const float2 old = o[p];
                val.x += old.x;
                val.y += old.y;
            }
            o[p] = val;
        }
    }
}

// One pass over the visibilities, pair by pair. A segment of L lanes (a power of two <= 64)
// takes one antenna pair: lanes stride over the channels of each of the pair's rows, a lane
// loading the npol values of one (row, channel) record at once. Modes:
//   0: (P, Q) of the pair against a model array (every polarisation);
//   1: (P, Q) against the source `next` (parallel hands; cross hands of an unpolarised
//      point source are zero);
//   2: first add G S e to the parallel hands of the record (the source `sub`, its flux
//      negated for a removal, times G = g[a1] conj(g[a2])) and write the record back, then
//      (P, Q) of the updated values against `next`;
//   3: the update of mode 2 only.
// The segment sums its lanes' (P, Q) by butterfly shuffles (fixed order). Each wave takes
// 64 / L pairs at a time and strides over the pairs.
struct PairArgs {
    float2 *vis;
    const float2 *model;
    const double *uvw, *kf;
    const Src *sub, *next;
    const float2 *gains;       // gains of the removed source (modes 2, 3)
    const uint32_t *pant;      // [npair] a1 | a2 << 16
    const int32_t *pstart;     // [npair + 1] CSR of each pair's rows
    const int32_t *prows;      // [nrow]
    const float *weights;      // [ngroups] or null
    int64_t npair;
    int nchan, npol, L;
    float4 *pq;                // [npair] (Re P, Im P, Q, 0)
};

template <int NPOL>
__device__ inline void load_rec(const float2 *src, float2 (&v)[4]) {
    if constexpr (NPOL == 4) {
        const float4 x = ((const float4 *)src)[0], y = ((const float4 *)src)[1];
        v[0] = make_float2(x.x, x.y);
        v[1] = make_float2(x.z, x.w);
        v[2] = make_float2(y.x, y.y);
        v[3] = make_float2(y.z, y.w);
    } else if constexpr (NPOL == 2) {
        const float4 x = ((const float4 *)src)[0];
        v[0] = make_float2(x.x, x.y);
        v[1] = make_float2(x.z, x.w);
    } else {
        v[0] = src[0];
    }
}

template <int NPOL>
__device__ inline void store_rec(float2 *dst, const float2 (&v)[4]) {
    if constexpr (NPOL == 4) {
        ((float4 *)dst)[0] = make_float4(v[0].x, v[0].y, v[1].x, v[1].y);
        ((float4 *)dst)[1] = make_float4(v[2].x, v[2].y, v[3].x, v[3].y);
    } else if constexpr (NPOL == 2) {
        ((float4 *)dst)[0] = make_float4(v[0].x, v[0].y, v[1].x, v[1].y);
    } else {
        dst[0] = v[0];
    }
}

template <int MODE, int NPOL>
__global__ __launch_bounds__(kBlock) void k_cal_pairs(PairArgs a) {
    const int lane = (int)(threadIdx.x & 63);
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int L = a.L, spw = 64 / L, seg = lane / L, sl = lane % L;
    constexpr bool SUB = MODE >= 2, MEASURE = MODE <= 2;
    Src sn{}, ss{};
    if constexpr (MODE == 1 || MODE == 2) sn = *a.next;
    if constexpr (SUB) ss = *a.sub;
    for (int64_t b0 = wave * spw; b0 < a.npair; b0 += nwave * spw) {
        const int64_t b = b0 + seg;
        const bool live = b < a.npair;
        float pr = 0.f, pi = 0.f, q = 0.f;
        if (live) {
            float gr = 0.f, gi = 0.f;  // g[a1] conj(g[a2])
            if constexpr (SUB) {
                const uint32_t an = a.pant[b];
                const float2 g1 = a.gains[an & 0xFFFFu], g2 = a.gains[an >> 16];
                gr = g1.x * g2.x + g1.y * g2.y;
                gi = g1.y * g2.x - g1.x * g2.y;
            }
            const int k1 = a.pstart[b + 1];
            for (int k = a.pstart[b]; k < k1; k++) {
                const int64_t r = a.prows[k];
                double path_s = 0.0, path_n = 0.0;
                if constexpr (SUB) path_s = a.uvw[3 * r] * ss.l + a.uvw[3 * r + 1] * ss.m + a.uvw[3 * r + 2] * ss.n1;
                if constexpr (MODE == 1 || MODE == 2)
                    path_n = a.uvw[3 * r] * sn.l + a.uvw[3 * r + 1] * sn.m + a.uvw[3 * r + 2] * sn.n1;
                for (int c = sl; c < a.nchan; c += L) {
                    const int64_t g = r * a.nchan + c;
                    float2 *rec = a.vis + g * NPOL;
                    float2 v[4];
                    load_rec<NPOL>(rec, v);
                    const double k = a.kf[c];
                    if constexpr (SUB) {
                        const float2 e = turn_phasor(path_s * k);
                        const float sr = (float)ss.flux * e.x, si = (float)ss.flux * e.y;
                        const float tr = gr * sr - gi * si, ti = gr * si + gi * sr;
#pragma unroll
                        for (int p = 0; p < NPOL; p++) {
                            if (NPOL == 4 && (p == 1 || p == 2)) continue;
                            v[p].x += tr;
                            v[p].y += ti;
                        }
                        store_rec<NPOL>(rec, v);
                    }
                    if constexpr (MEASURE) {
                        const float wt = a.weights ? a.weights[g] : 1.0f;
                        if (wt != 0.0f) {
                            if constexpr (MODE == 0) {
                                float2 m[4];
                                load_rec<NPOL>(a.model + g * NPOL, m);
#pragma unroll
                                for (int p = 0; p < NPOL; p++) {
                                    pr += wt * (m[p].x * v[p].x + m[p].y * v[p].y);
                                    pi += wt * (m[p].x * v[p].y - m[p].y * v[p].x);
                                    q += wt * (m[p].x * m[p].x + m[p].y * m[p].y);
                                }
                            } else {
                                const float2 e = turn_phasor(path_n * k);
                                const float mx = (float)sn.flux * e.x, my = (float)sn.flux * e.y;
#pragma unroll
                                for (int p = 0; p < NPOL; p++) {
                                    if (NPOL == 4 && (p == 1 || p == 2)) continue;
                                    pr += wt * (mx * v[p].x + my * v[p].y);
                                    pi += wt * (mx * v[p].y - my * v[p].x);
                                    q += wt * (mx * mx + my * my);
                                }
                            }
                        }
                    }
                }
            }
        }
        if constexpr (MEASURE) {
            for (int o = L / 2; o >= 1; o >>= 1) {
                pr += __shfl_xor(pr, o, 64);
                pi += __shfl_xor(pi, o, 64);
                q += __shfl_xor(q, o, 64);
            }
            if (live && sl == 0) a.pq[b] = make_float4(pr, pi, q, 0.f);
        }
    }
}

// f / c of every channel (FP64 division, correctly rounded like the host's)
__global__ void k_turns_per_metre(const double *freq, int n, double *kf) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) kf[i] = freq[i] / kC;
}

__global__ void k_fill_gains(float2 *g, int n, float2 v) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) g[i] = v;
}

// One StEFCal iteration (number it, from 1): one workgroup per antenna gathers its pairs'
// (P, Q) (FP64 sums: each thread a strided share of the list, then a fixed-order tree), solves
// its gain and writes the next iterate (the mean with the previous one on even iterations);
// diff / nrm receive |g_new - g_old|^2 and |g_new|^2. A whole workgroup per antenna keeps
// many independent loads of the list in flight.
__global__ __launch_bounds__(kBlock) void k_cal_ants(const float4 *pq, const int32_t *partner, const int32_t *start,
                                                     const int32_t *entry, int nant, const float2 *gin, float2 *gout,
                                                     int it, double *diff, double *nrm) {
    __shared__ double sr[kBlock], si[kBlock], sd[kBlock];
    const int t = (int)threadIdx.x;
    const int a = (int)blockIdx.x;
    double nr = 0, ni = 0, dd = 0;
#pragma unroll 4
    for (int k = start[a] + t; k < start[a + 1]; k += kBlock) {
        const int32_t e = entry[k];
        const float4 v = pq[e >> 1];
        const float2 o = gin[partner[k]];
        // a1(b) = a: g[a2] P; a2(b) = a: g[a1] conj(P)
        const double pim = (e & 1) ? -(double)v.y : (double)v.y;
        nr += (double)o.x * v.x - (double)o.y * pim;
        ni += (double)o.x * pim + (double)o.y * v.x;
        dd += ((double)o.x * o.x + (double)o.y * o.y) * v.z;
    }
    sr[t] = nr;
    si[t] = ni;
    sd[t] = dd;
    __syncthreads();
    for (int o = kBlock / 2; o >= 1; o >>= 1) {
        if (t < o) {
            sr[t] += sr[t + o];
            si[t] += si[t + o];
            sd[t] += sd[t + o];
        }
        __syncthreads();
    }
    if (t == 0) {
        const float2 old = gin[a];
        double gr = old.x, gi = old.y;
        if (sd[0] > 0.0) {
            gr = sr[0] / sd[0];
            gi = si[0] / sd[0];
        }
        const double dr = gr - old.x, di = gi - old.y;
        if (diff) {
            diff[a] = dr * dr + di * di;
            nrm[a] = gr * gr + gi * gi;
        }
        if ((it & 1) == 0) {
            gr = 0.5 * (gr + old.x);
            gi = 0.5 * (gi + old.y);
        }
        gout[a] = make_float2((float)gr, (float)gi);
    }
}

// rel = sqrt(sum diff / sum nrm) over the antennas (one workgroup, fixed order), optionally
// also copying the gains to their destination.
__global__ __launch_bounds__(kBlock) void k_cal_finish(const double *diff, const double *nrm, int nant, float *rel,
                                                       const float2 *g, float2 *gdst) {
    __shared__ double sd[kBlock], sn[kBlock];
    const int t = (int)threadIdx.x;
    double a = 0, b = 0;
    for (int i = t; i < nant; i += kBlock) {
        if (diff) {
            a += diff[i];
            b += nrm[i];
        }
        if (gdst) gdst[i] = g[i];
    }
    sd[t] = a;
    sn[t] = b;
    __syncthreads();
    for (int o = kBlock / 2; o >= 1; o >>= 1) {
        if (t < o) {
            sd[t] += sd[t + o];
            sn[t] += sn[t + o];
        }
        __syncthreads();
    }
    if (t == 0 && rel) *rel = sn[0] > 0 ? (float)sqrt(sd[0] / sn[0]) : 0.f;
}

__global__ void k_stage_sources(const double *src, int nsrc, Src *out) {
    const int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (k >= nsrc) return;
    const double l = src[3 * k], m = src[3 * k + 1];
    out[k] = {l, m, sqrt(fmax(0.0, 1.0 - l * l - m * m)) - 1.0, src[3 * k + 2]};
}

int lanes_per_row(int ne) {
    int L = 1;
    while (L < ne && L < 64) L *= 2;
    return L;
}

// One pass of k_cal_pairs in the given mode (see there).
Status cal_pass(Instance &I, int mode, float2 *vis, const float2 *model, const Src *sub, const Src *next,
                const float2 *gains, const float *weights, hipStream_t s) {
    if (I.cal_npair == 0) return Status::Ok();
    PairArgs a;
    a.vis = vis;
    a.model = model;
    a.uvw = I.uvw_d;
    a.kf = I.kf_d;
    a.sub = sub;
    a.next = next;
    a.gains = gains;
    a.pant = I.cal_pant;
    a.pstart = I.cal_pstart;
    a.prows = I.cal_prows;
    a.weights = weights;
    a.npair = I.cal_npair;
    a.nchan = I.nchan;
    a.npol = I.npol;
    a.L = lanes_per_row(I.nchan);
    a.pq = I.cal_pq;
    const int64_t waves = (I.cal_npair + (64 / a.L) - 1) / (64 / a.L);
    // about 4 rounds of pairs per wave, at most 2048 workgroups
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(2048, (waves + 15) / 16));
#define MWG_PASS(M, NP) hipLaunchKernelGGL((k_cal_pairs<M, NP>), dim3(blocks), dim3(kBlock), 0, s, a)
#define MWG_PASS_NP(M)                                                                                        \
    do {                                                                                                      \
        if (I.npol == 4) MWG_PASS(M, 4);                                                                      \
        else if (I.npol == 2) MWG_PASS(M, 2);                                                                 \
        else MWG_PASS(M, 1);                                                                                  \
    } while (0)
    switch (mode) {
    case 0: MWG_PASS_NP(0); break;
    case 1: MWG_PASS_NP(1); break;
    case 2: MWG_PASS_NP(2); break;
    default: MWG_PASS_NP(3); break;
    }
#undef MWG_PASS_NP
#undef MWG_PASS
    MWG_HIP(hipGetLastError());
    return Status::Ok();
}

// niter iterations from the gains in g (device [nant]) on the pairs' (P, Q) of the last
// pass; the solution ends in g, the last iteration's relative step in *rel (device) when
// rel is given.
Status iterate(Instance &I, float2 *g, int niter, float *rel, hipStream_t s) {
    // ping-pong between g and the plan's second gain buffer, ending in g
    float2 *bufs[2] = {g, I.cal_g};
    int cur = 0;
    if (niter % 2 == 1) {  // start from the second buffer so that the last iterate lands in g
        MWG_HIP(hipMemcpyAsync(I.cal_g, g, sizeof(float2) * (size_t)I.nant, hipMemcpyDeviceToDevice, s));
        cur = 1;
    }
    for (int it = 1; it <= niter; it++) {
        const bool last = it == niter;
        hipLaunchKernelGGL(k_cal_ants, dim3((unsigned)I.nant), dim3(kBlock), 0, s, I.cal_pq,
                           I.cal_partner, I.cal_start, I.cal_entry, I.nant, bufs[cur], bufs[cur ^ 1], it,
                           last && rel ? I.cal_red : nullptr, I.cal_red + I.nant);
        MWG_HIP(hipGetLastError());
        cur ^= 1;
    }
    if (rel) {  // (no iteration: a step of 0)
        hipLaunchKernelGGL(k_cal_finish, dim3(1), dim3(kBlock), 0, s, niter > 0 ? I.cal_red : nullptr,
                           I.cal_red + I.nant, I.nant, rel, nullptr, nullptr);
        MWG_HIP(hipGetLastError());
    }
    return Status::Ok();
}

// Antenna-pair lists on the device (up to 2048 antennas: a dense table of pair keys
// a1 * nant + a2). The pairs are numbered in order of their first row: each key's first row by
// an atomic minimum, then a scan over the rows that are first of their key.
__global__ void k_pair_first(const int32_t *a1, const int32_t *a2, int64_t nrow, int nant, uint32_t *first) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < nrow) atomicMin(&first[(uint32_t)a1[r] * (uint32_t)nant + (uint32_t)a2[r]], (uint32_t)r);
}

__global__ void k_pair_flag(const int32_t *a1, const int32_t *a2, int64_t nrow, int nant, const uint32_t *first,
                            uint32_t *flag) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < nrow) flag[r] = first[(uint32_t)a1[r] * (uint32_t)nant + (uint32_t)a2[r]] == (uint32_t)r ? 1u : 0u;
}

// pair of every row; the first row of each pair writes the pair's antennas
__global__ void k_pair_ids(const int32_t *a1, const int32_t *a2, int64_t nrow, int nant, const uint32_t *first,
                           const uint32_t *scan, uint32_t *pair_of, uint32_t *pant) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrow) return;
    const uint32_t f = first[(uint32_t)a1[r] * (uint32_t)nant + (uint32_t)a2[r]], pid = scan[f];
    pair_of[r] = pid;
    if (f == (uint32_t)r) pant[pid] = (uint32_t)a1[r] | (uint32_t)a2[r] << 16;
}

// first index of every pair in the pair-sorted rows (every pair has a row), and the end
__global__ void k_pair_starts(const uint32_t *skeys, int64_t n, int64_t npair, int32_t *pstart) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (i == 0 || skeys[i - 1] != skeys[i]) pstart[skeys[i]] = (int32_t)i;
    if (i == n - 1) pstart[npair] = (int32_t)n;
}

// entry e = pair << 1 | side belongs to the pair's first (side 0) or second antenna
__global__ void k_ant_keys(const uint32_t *pant, int64_t nent, uint32_t *keys, uint32_t *counts) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nent) return;
    const uint32_t p = pant[e >> 1], a = (e & 1) ? p >> 16 : p & 0xFFFFu;
    keys[e] = a;
    atomicAdd(&counts[a], 1u);
}

__global__ void k_ant_lists(const uint32_t *sorted_e, const uint32_t *pant, int64_t nent, int32_t *entry,
                            int32_t *partner) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nent) return;
    const uint32_t e = sorted_e[k], p = pant[e >> 1];
    entry[k] = (int32_t)e;
    partner[k] = (int32_t)((e & 1) ? (p & 0xFFFFu) : (p >> 16));
}

int bits_for(uint64_t maxval) {
    int r = 1;
    while (r < 32 && (maxval >> r) != 0) r++;
    return r;
}

} // namespace

Status sort_pairs(uint32_t *keys, uint32_t *keys_alt, const uint32_t *vals_init, uint32_t *vals,
                  uint32_t *vals_alt, int64_t n, int keybits, uint32_t **keys_out, uint32_t **vals_out,
                  hipStream_t s);
Status exclusive_scan_u32(uint32_t *data, int64_t n, hipStream_t s);
Status launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);

Status stage_sources(Instance &I, const double *sources, int nsrc, bool from_host, hipStream_t s);

// Plan-time state of prediction and calibration: device copies of uvw and f / c, and (with
// antennas) the antenna pairs: each pair's rows, each antenna's pairs, the per-pair sums and
// the gain buffers. Pairs are numbered in order of their first row; an antenna's pairs and a
// pair's rows are listed in ascending order.
Status build_calibration(Instance &I, const double *uvw_dev, const double *freq_dev, const int32_t *a1_dev,
                         const int32_t *a2_dev, hipStream_t s) {
    void *p;
    MWG_TRY(I.arena.alloc(&p, sizeof(double) * 3 * (size_t)std::max<int64_t>(I.nrow, 1)));
    I.uvw_d = (double *)p;
    if (I.nrow > 0)
        MWG_HIP(hipMemcpyAsync(I.uvw_d, uvw_dev, sizeof(double) * 3 * (size_t)I.nrow, hipMemcpyDeviceToDevice, s));
    MWG_TRY(I.arena.alloc(&p, sizeof(double) * (size_t)std::max(I.nchan, 1)));
    I.kf_d = (double *)p;
    hipLaunchKernelGGL(k_turns_per_metre, dim3(grid1d(I.nchan)), dim3(kBlock), 0, s, freq_dev, I.nchan, I.kf_d);
    MWG_HIP(hipGetLastError());
    if (!I.has_ants) return Status::Ok();
    if (I.nrow >= (int64_t)1 << 30) return make_error(MW_ERR_UNSUPPORTED, "calibration lists need nrow < 2^30");
    auto alloc_lists = [&](int64_t npair) -> Status {
        I.cal_npair = npair;
        MWG_TRY(I.arena.alloc(&p, 4 * ((size_t)I.nant + 1)));
        I.cal_start = (int32_t *)p;
        MWG_TRY(I.arena.alloc(&p, 4 * std::max<size_t>(2 * (size_t)npair, 1)));
        I.cal_entry = (int32_t *)p;
        MWG_TRY(I.arena.alloc(&p, 4 * std::max<size_t>(2 * (size_t)npair, 1)));
        I.cal_partner = (int32_t *)p;
        MWG_TRY(I.arena.alloc(&p, 4 * std::max<size_t>((size_t)npair, 1)));
        I.cal_pant = (uint32_t *)p;
        MWG_TRY(I.arena.alloc(&p, 4 * ((size_t)npair + 1)));
        I.cal_pstart = (int32_t *)p;
        MWG_TRY(I.arena.alloc(&p, 4 * std::max<size_t>((size_t)I.nrow, 1)));
        I.cal_prows = (int32_t *)p;
        MWG_TRY(I.arena.alloc(&p, sizeof(float4) * (size_t)std::max<int64_t>(npair, 1)));
        I.cal_pq = (float4 *)p;
        MWG_TRY(I.arena.alloc(&p, sizeof(float2) * (size_t)I.nant));
        I.cal_g = (float2 *)p;
        MWG_TRY(I.arena.alloc(&p, sizeof(double) * 2 * (size_t)I.nant));
        I.cal_red = (double *)p;
        return Status::Ok();
    };
    const int64_t nn = (int64_t)I.nant * I.nant;
    if (nn <= ((int64_t)1 << 22)) {
        // on the device: pair numbers, each pair's rows (a stable sort of the rows by pair) and
        // each antenna's pairs (a stable sort of the entries by antenna), as the host lists
        // below would give them
        const int64_t nrow = I.nrow;
        if (nrow == 0) {
            MWG_TRY(alloc_lists(0));
            MWG_TRY(launch_fill_u32((uint32_t *)I.cal_start, I.nant + 1, 0u, s));
            MWG_TRY(launch_fill_u32((uint32_t *)I.cal_pstart, 1, 0u, s));
            return Status::Ok();
        }
        DevTmp first, flag;
        MWG_TRY(first.alloc(4 * (size_t)nn, s));
        MWG_TRY(flag.alloc(4 * ((size_t)nrow + 1), s));
        MWG_TRY(launch_fill_u32(first.as<uint32_t>(), nn, 0xFFFFFFFFu, s));
        MWG_TRY(launch_fill_u32(flag.as<uint32_t>() + nrow, 1, 0u, s));
        hipLaunchKernelGGL(k_pair_first, dim3(grid1d(nrow)), dim3(kBlock), 0, s, a1_dev, a2_dev, nrow, I.nant,
                           first.as<uint32_t>());
        hipLaunchKernelGGL(k_pair_flag, dim3(grid1d(nrow)), dim3(kBlock), 0, s, a1_dev, a2_dev, nrow, I.nant,
                           first.as<uint32_t>(), flag.as<uint32_t>());
        MWG_HIP(hipGetLastError());
        MWG_TRY(exclusive_scan_u32(flag.as<uint32_t>(), nrow + 1, s));
        uint32_t hnpair = 0;
        MWG_HIP(hipMemcpyAsync(&hnpair, flag.as<uint32_t>() + nrow, 4, hipMemcpyDeviceToHost, s));
        MWG_HIP(hipStreamSynchronize(s));
        const int64_t npair = hnpair;
        MWG_TRY(alloc_lists(npair));
        // rows of each pair
        DevTmp keys, keys2, vals, vals2;
        MWG_TRY(keys.alloc(4 * (size_t)nrow, s));
        MWG_TRY(keys2.alloc(4 * (size_t)nrow, s));
        MWG_TRY(vals.alloc(4 * (size_t)nrow, s));
        MWG_TRY(vals2.alloc(4 * (size_t)nrow, s));
        hipLaunchKernelGGL(k_pair_ids, dim3(grid1d(nrow)), dim3(kBlock), 0, s, a1_dev, a2_dev, nrow, I.nant,
                           first.as<uint32_t>(), flag.as<uint32_t>(), keys.as<uint32_t>(), I.cal_pant);
        MWG_HIP(hipGetLastError());
        uint32_t *sk = nullptr, *sv = nullptr;
        MWG_TRY(sort_pairs(keys.as<uint32_t>(), keys2.as<uint32_t>(), nullptr, vals.as<uint32_t>(),
                           vals2.as<uint32_t>(), nrow, bits_for((uint64_t)npair - 1), &sk, &sv, s));
        MWG_HIP(hipMemcpyAsync(I.cal_prows, sv, 4 * (size_t)nrow, hipMemcpyDeviceToDevice, s));
        hipLaunchKernelGGL(k_pair_starts, dim3(grid1d(nrow)), dim3(kBlock), 0, s, sk, nrow, npair, I.cal_pstart);
        MWG_HIP(hipGetLastError());
        // pairs of each antenna
        const int64_t nent = 2 * npair;
        DevTmp ek, ek2, ev, ev2, counts;
        MWG_TRY(ek.alloc(4 * (size_t)nent, s));
        MWG_TRY(ek2.alloc(4 * (size_t)nent, s));
        MWG_TRY(ev.alloc(4 * (size_t)nent, s));
        MWG_TRY(ev2.alloc(4 * (size_t)nent, s));
        MWG_TRY(counts.alloc(4 * ((size_t)I.nant + 1), s));
        MWG_TRY(launch_fill_u32(counts.as<uint32_t>(), I.nant + 1, 0u, s));
        hipLaunchKernelGGL(k_ant_keys, dim3(grid1d(nent)), dim3(kBlock), 0, s, I.cal_pant, nent, ek.as<uint32_t>(),
                           counts.as<uint32_t>());
        MWG_HIP(hipGetLastError());
        MWG_TRY(exclusive_scan_u32(counts.as<uint32_t>(), I.nant + 1, s));
        MWG_HIP(hipMemcpyAsync(I.cal_start, counts.p, 4 * ((size_t)I.nant + 1), hipMemcpyDeviceToDevice, s));
        uint32_t *esk = nullptr, *esv = nullptr;
        MWG_TRY(sort_pairs(ek.as<uint32_t>(), ek2.as<uint32_t>(), nullptr, ev.as<uint32_t>(), ev2.as<uint32_t>(),
                           nent, bits_for((uint64_t)I.nant - 1), &esk, &esv, s));
        hipLaunchKernelGGL(k_ant_lists, dim3(grid1d(nent)), dim3(kBlock), 0, s, esv, I.cal_pant, nent, I.cal_entry,
                           I.cal_partner);
        MWG_HIP(hipGetLastError());
        if (!first.pooled()) MWG_HIP(hipStreamSynchronize(s));  // temporaries outlive the kernels
        return Status::Ok();
    }
    std::vector<int32_t> h1((size_t)I.nrow), h2((size_t)I.nrow);
    if (I.nrow > 0) {
        MWG_HIP(hipMemcpyAsync(h1.data(), a1_dev, 4 * (size_t)I.nrow, hipMemcpyDeviceToHost, s));
        MWG_HIP(hipMemcpyAsync(h2.data(), a2_dev, 4 * (size_t)I.nrow, hipMemcpyDeviceToHost, s));
    }
    MWG_HIP(hipStreamSynchronize(s));
    // more than 2048 antennas: the pair of every row from a hash map, on the host
    std::vector<int32_t> pair_of((size_t)I.nrow);
    std::vector<uint32_t> pant;
    {
        std::unordered_map<uint64_t, int32_t> id;
        for (int64_t r = 0; r < I.nrow; r++) {
            auto ins = id.emplace((uint64_t)h1[r] << 32 | (uint32_t)h2[r], (int32_t)pant.size());
            if (ins.second) pant.push_back((uint32_t)h1[r] | (uint32_t)h2[r] << 16);
            pair_of[r] = ins.first->second;
        }
    }
    const int64_t npair = (int64_t)pant.size();
    // rows of each pair
    std::vector<int32_t> pstart((size_t)npair + 1, 0), prows((size_t)I.nrow);
    for (int64_t r = 0; r < I.nrow; r++) pstart[pair_of[r] + 1]++;
    for (int64_t b = 0; b < npair; b++) pstart[b + 1] += pstart[b];
    {
        std::vector<int32_t> fill(pstart.begin(), pstart.end() - 1);
        for (int64_t r = 0; r < I.nrow; r++) prows[fill[pair_of[r]]++] = (int32_t)r;
    }
    // pairs of each antenna: entry = pair << 1 | (0: as ant1, 1: as ant2), partner = the other
    std::vector<int32_t> start((size_t)I.nant + 1, 0), entry(2 * (size_t)npair), partner(2 * (size_t)npair);
    for (int64_t b = 0; b < npair; b++) {
        start[(pant[b] & 0xFFFFu) + 1]++;
        start[(pant[b] >> 16) + 1]++;
    }
    for (int a = 0; a < I.nant; a++) start[a + 1] += start[a];
    {
        std::vector<int32_t> fill(start.begin(), start.end() - 1);
        for (int64_t b = 0; b < npair; b++) {
            const int a1 = (int)(pant[b] & 0xFFFFu), a2 = (int)(pant[b] >> 16);
            partner[fill[a1]] = a2;
            entry[fill[a1]++] = (int32_t)(b << 1);
            partner[fill[a2]] = a1;
            entry[fill[a2]++] = (int32_t)(b << 1 | 1);
        }
    }
    MWG_TRY(alloc_lists(npair));
    MWG_HIP(hipMemcpyAsync(I.cal_start, start.data(), 4 * start.size(), hipMemcpyHostToDevice, s));
    MWG_HIP(hipMemcpyAsync(I.cal_pstart, pstart.data(), 4 * pstart.size(), hipMemcpyHostToDevice, s));
    if (npair > 0) {
        MWG_HIP(hipMemcpyAsync(I.cal_entry, entry.data(), 4 * entry.size(), hipMemcpyHostToDevice, s));
        MWG_HIP(hipMemcpyAsync(I.cal_partner, partner.data(), 4 * partner.size(), hipMemcpyHostToDevice, s));
        MWG_HIP(hipMemcpyAsync(I.cal_pant, pant.data(), 4 * pant.size(), hipMemcpyHostToDevice, s));
        MWG_HIP(hipMemcpyAsync(I.cal_prows, prows.data(), 4 * prows.size(), hipMemcpyHostToDevice, s));
    }
    MWG_HIP(hipStreamSynchronize(s));
    return Status::Ok();
}

Status launch_predict(Instance &I, const double *sources, int nsrc, const float2 *gains, float2 *out,
                      int accumulate, hipStream_t s) {
    if (I.ngroups == 0) return Status::Ok();
    if (nsrc < 0) return make_error(MW_ERR_INVALID_ARG, "nsrc must be >= 0");
    if (gains && !I.has_ants) return make_error(MW_ERR_STATE, "gains given for an instance planned without antennas");
    // the source table as (l, m, n - 1, S) in the plan's device buffer
    MWG_TRY(stage_sources(I, sources, nsrc, false, s));
    const int64_t nthreads = I.nrow * ((I.nchan + kPredChan - 1) / kPredChan);
    hipLaunchKernelGGL(k_predict, dim3(grid1d(nthreads)), dim3(kBlock), 0, s, I.uvw_d, I.kf_d, I.nrow, I.nchan,
                       I.npol, (const Src *)I.src_d, nsrc, gains, I.ant_orig, out, accumulate);
    MWG_HIP(hipGetLastError());
    return Status::Ok();
}

Status launch_solve_gains(Instance &I, const float2 *vis, const float2 *model, const float *weights, float2 *gains,
                          int niter, float *rel, hipStream_t s) {
    if (!I.has_ants) return make_error(MW_ERR_STATE, "gain solving needs an instance planned with antennas");
    if (niter < 0) return make_error(MW_ERR_INVALID_ARG, "niter must be >= 0");
    MWG_TRY(cal_pass(I, 0, const_cast<float2 *>(vis), model, nullptr, nullptr, nullptr, weights, s));
    return iterate(I, gains, niter, rel, s);
}

Status launch_peel(Instance &I, const float2 *vis, const double *sources_host, int nsrc, const float *weights,
                   int niter, float2 *resid, float2 *gains, float *rel, hipStream_t s) {
    if (!I.has_ants) return make_error(MW_ERR_STATE, "peeling needs an instance planned with antennas");
    if (niter < 1 || nsrc < 0) return make_error(MW_ERR_INVALID_ARG, "niter must be >= 1 and nsrc >= 0");
    const size_t nbytes = sizeof(float2) * (size_t)I.ngroups * I.npol;
    if (resid != vis && nbytes > 0) MWG_HIP(hipMemcpyAsync(resid, vis, nbytes, hipMemcpyDeviceToDevice, s));
    if (nsrc == 0) return Status::Ok();
    // decreasing |S|, ties in catalogue order; each source also in negated form for removal
    std::vector<int> order((size_t)nsrc);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return std::fabs(sources_host[3 * (size_t)x + 2]) > std::fabs(sources_host[3 * (size_t)y + 2]);
    });
    MWG_TRY(stage_sources(I, sources_host, nsrc, true, s));
    const Src *table = (const Src *)I.src_d;  // [2 nsrc]: source k, then its negation at nsrc + k
    // pass i: remove source order[i - 1] with its gains (from the second source on) and form
    // (P, Q) of order[i]; a last pass removes the last source
    for (size_t i = 0; i < order.size(); i++) {
        const int k = order[i];
        float2 *gk = gains + (size_t)k * I.nant;
        hipLaunchKernelGGL(k_fill_gains, dim3(grid1d(I.nant)), dim3(kBlock), 0, s, gk, I.nant, make_float2(1.f, 0.f));
        MWG_HIP(hipGetLastError());
        if (i == 0) {
            MWG_TRY(cal_pass(I, 1, resid, nullptr, nullptr, table + k, nullptr, weights, s));
        } else {
            const int kp = order[i - 1];
            MWG_TRY(cal_pass(I, 2, resid, nullptr, table + nsrc + kp, table + k, gains + (size_t)kp * I.nant, weights,
                             s));
        }
        MWG_TRY(iterate(I, gk, niter, rel ? rel + k : nullptr, s));
    }
    const int kl = order.back();
    MWG_TRY(cal_pass(I, 3, resid, nullptr, table + nsrc + kl, nullptr, gains + (size_t)kl * I.nant, nullptr, s));
    return Status::Ok();
}

// Copies a source table (l, m, S rows; host, or device when from_host is false) into the
// plan's device buffer as (l, m, n - 1, S), followed, for peeling, by the negated sources.
Status stage_sources(Instance &I, const double *sources, int nsrc, bool from_host, hipStream_t s) {
    const size_t need = (size_t)std::max(nsrc, 1) * (from_host ? 2 : 1);
    if (I.src_cap < need) {
        void *p;
        MWG_TRY(I.arena.alloc(&p, sizeof(Src) * need));
        I.src_d = p;
        I.src_cap = need;
        if (I.src_h) (void)hipHostFree(I.src_h);
        I.src_h = nullptr;
        if (hipHostMalloc(&I.src_h, sizeof(Src) * need, hipHostMallocDefault) != hipSuccess) {
            I.src_h = nullptr;
            return make_error(MW_ERR_ALLOC, "hipHostMalloc of the source table failed");
        }
    }
    if (nsrc == 0) return Status::Ok();
    if (!from_host) {
        // device table: (l, m, S) -> (l, m, n - 1, S) on the device
        hipLaunchKernelGGL(k_stage_sources, dim3(grid1d(nsrc)), dim3(kBlock), 0, s, sources, nsrc, (Src *)I.src_d);
        MWG_HIP(hipGetLastError());
        return Status::Ok();
    }
    if (I.src_pending) {
        MWG_HIP(hipEventSynchronize(I.src_ev));  // the previous upload has read the pinned table
        I.src_pending = false;
    }
    Src *h = (Src *)I.src_h;
    for (int k = 0; k < nsrc; k++) {
        const double l = sources[3 * (size_t)k], m = sources[3 * (size_t)k + 1], S = sources[3 * (size_t)k + 2];
        const double n1 = std::sqrt(std::max(0.0, 1.0 - l * l - m * m)) - 1.0;
        h[k] = {l, m, n1, S};
        h[nsrc + k] = {l, m, n1, -S};
    }
    MWG_HIP(hipMemcpyAsync(I.src_d, I.src_h, sizeof(Src) * 2 * (size_t)nsrc, hipMemcpyHostToDevice, s));
    if (!I.src_ev) MWG_HIP(hipEventCreateWithFlags(&I.src_ev, hipEventDisableTiming));
    MWG_HIP(hipEventRecord(I.src_ev, s));
    I.src_pending = true;
    return Status::Ok();
}

} // namespace mwg
