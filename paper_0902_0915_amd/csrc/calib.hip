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
// one. With scalar gains, every sample of one row (one baseline at one time) has the same
// antenna pair, so the sums factor through two per-row numbers that do not depend on g:
//     P_r = sum_{chan, pol} w conj(M) V,    Q_r = sum w |M|^2.
// Antenna p then needs num_p = sum_{a1(r) = p} g[a2] P_r + sum_{a2(r) = p} g[a1] conj(P_r) and
// den_p = sum_{a1 = p} |g[a2]|^2 Q_r + sum_{a2 = p} |g[a1]|^2 Q_r. One pass over the
// visibilities forms (P, Q); every iteration after that reads only the rows' (P, Q) through a
// per-antenna list of rows built with the plan, so the iterations cost almost nothing.
//
// Peeling. For each source in decreasing |S| (ties in catalogue order): (P, Q) of the current
// residual against the source's prediction, the iterations from unit gains, then the
// residual minus g[a1] conj(g[a2]) times the prediction. Everything is enqueued on the
// caller's stream; the only host work is ordering the catalogue.
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

namespace mwg {

namespace {

constexpr double kC = 299792458.0;
constexpr int kBlock = 256;

unsigned grid1d(int64_t n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

// exp(-2 pi i t) for t in turns (FP64), evaluated after reduction to [-1/2, 1/2] turn
__device__ inline float2 turn_phasor(double t) {
    const double fr = t - rint(t);
    float s, c;
    sincospif(-2.0f * (float)fr, &s, &c);
    return make_float2(c, s);
}

struct Src {
    double l, m, n1, flux;  // n1 = sqrt(1 - l^2 - m^2) - 1
};

// Model visibilities of nsrc point sources (sources in global memory, read through L1), times
// g[a1] conj(g[a2]) when gains are given; written or added to out [ng][npol]. Cross
// polarisations (1, 2 of 4) of an unpolarised source are zero. One thread per group.
__global__ __launch_bounds__(kBlock) void k_predict(const double *uvw, const double *kf, int64_t ng, int nchan,
                                                    int npol, const Src *src, int nsrc, const float2 *gains,
                                                    const uint32_t *ants, float2 *out, int accumulate) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ng) return;
    const uint32_t r = (uint32_t)g / (uint32_t)nchan;  // ngroups < 2^31
    const int c = (int)((uint32_t)g - r * (uint32_t)nchan);
    const double k = kf[c];  // turns per metre, f / c
    const double u = uvw[3 * r], v = uvw[3 * r + 1], w = uvw[3 * r + 2];
    float sr = 0.f, si = 0.f;
    for (int j = 0; j < nsrc; j++) {
        const Src q = src[j];
        const double path = u * q.l + v * q.m + w * q.n1;
        const float2 e = turn_phasor(path * k);
        sr += (float)q.flux * e.x;
        si += (float)q.flux * e.y;
    }
    if (gains) {
        const uint32_t an = ants[r];
        const float2 g1 = gains[an & 0xFFFFu], g2 = gains[an >> 16];
        const float gr = g1.x * g2.x + g1.y * g2.y, gi = g1.y * g2.x - g1.x * g2.y;  // g1 conj(g2)
        const float tr = gr * sr - gi * si, ti = gr * si + gi * sr;
        sr = tr;
        si = ti;
    }
    float2 *o = out + g * npol;
    for (int p = 0; p < npol; p++) {
        const bool cross = npol == 4 && (p == 1 || p == 2);
        float2 val = cross ? make_float2(0.f, 0.f) : make_float2(sr, si);
        if (accumulate) {
            const float2 old = o[p];
            val.x += old.x;
            val.y += old.y;
        }
        o[p] = val;
    }
}

// Per-row (P, Q) against a model array or one predicted source. A segment of L lanes (a power
// of two <= 64) takes one row: lanes stride over its nchan * npol samples, then the segment
// sums its values by butterfly shuffles (fixed order). Each wave takes 64 / L rows at a time
// and strides over the rows, so that a wave does a useful amount of work.
template <bool FROM_SOURCE>
__global__ __launch_bounds__(kBlock) void k_cal_rows(const float2 *vis, const float2 *model, const double *uvw,
                                                     const double *kf, const Src *src, const float *weights,
                                                     int64_t nrow, int nchan, int npol, int L, float4 *pq) {
    const int lane = (int)(threadIdx.x & 63);
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int spw = 64 / L, seg = lane / L, sl = lane % L;
    const int pshift = npol == 4 ? 2 : (npol == 2 ? 1 : 0);
    const int ne = nchan * npol;
    Src s{};
    if constexpr (FROM_SOURCE) s = *src;
    for (int64_t r0 = wave * spw; r0 < nrow; r0 += nwave * spw) {
        const int64_t r = r0 + seg;
        const bool live = r < nrow;
        float pr = 0.f, pi = 0.f, q = 0.f;
        if (live) {
            double path = 0.0;
            if constexpr (FROM_SOURCE) path = uvw[3 * r] * s.l + uvw[3 * r + 1] * s.m + uvw[3 * r + 2] * s.n1;
            for (int e = sl; e < ne; e += L) {
                const int c = e >> pshift, p = e & (npol - 1);
                const int64_t g = r * nchan + c;
                const float wt = weights ? weights[g] : 1.0f;
                if (wt == 0.0f) continue;
                float2 M;
                if constexpr (FROM_SOURCE) {
                    const bool cross = npol == 4 && (p == 1 || p == 2);
                    if (cross) continue;
                    const float2 ph = turn_phasor(path * kf[c]);
                    M = make_float2((float)s.flux * ph.x, (float)s.flux * ph.y);
                } else {
                    M = model[g * npol + p];
                }
                const float2 V = vis[g * npol + p];
                // conj(M) V and |M|^2, weighted
                pr += wt * (M.x * V.x + M.y * V.y);
                pi += wt * (M.x * V.y - M.y * V.x);
                q += wt * (M.x * M.x + M.y * M.y);
            }
        }
        for (int o = L / 2; o >= 1; o >>= 1) {
            pr += __shfl_xor(pr, o, 64);
            pi += __shfl_xor(pi, o, 64);
            q += __shfl_xor(q, o, 64);
        }
        if (live && sl == 0) pq[r] = make_float4(pr, pi, q, 0.f);
    }
}

__global__ void k_fill_gains(float2 *g, int n, float2 v) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) g[i] = v;
}

// One StEFCal iteration (number it, from 1): one workgroup per antenna gathers its rows'
// (P, Q) (FP64 sums: each thread a strided share of the list, then a fixed-order tree), solves
// its gain and writes the next iterate (the mean with the previous one on even iterations);
// diff / nrm receive |g_new - g_old|^2 and |g_new|^2. A whole workgroup per antenna keeps
// many independent loads of the list in flight (an antenna has thousands of rows).
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
        // a1(r) = a: g[a2] P; a2(r) = a: g[a1] conj(P)
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

// Per-row sums, then niter iterations starting from the gains in g (device [nant]); the
// solution ends in g, the last iteration's relative step in *rel (device) when rel is given.
Status solve(Instance &I, const float2 *vis, const float2 *model, const Src *src, const float *weights, float2 *g,
             int niter, float *rel, hipStream_t s) {
    const int L = lanes_per_row(I.nchan * I.npol);
    const int64_t waves = (I.nrow + (64 / L) - 1) / (64 / L);
    // about 16 rounds of rows per wave, at most 2048 workgroups
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(2048, (waves + 63) / 64));
    if (I.nrow > 0) {
        if (src)
            hipLaunchKernelGGL(k_cal_rows<true>, dim3(blocks), dim3(kBlock), 0, s, vis, model, I.uvw_d, I.kf_d, src,
                               weights, I.nrow, I.nchan, I.npol, L, I.cal_pq);
        else
            hipLaunchKernelGGL(k_cal_rows<false>, dim3(blocks), dim3(kBlock), 0, s, vis, model, I.uvw_d, I.kf_d, src,
                               weights, I.nrow, I.nchan, I.npol, L, I.cal_pq);
        MWG_HIP(hipGetLastError());
    }
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

} // namespace

Status stage_sources(Instance &I, const double *sources, int nsrc, bool from_host, hipStream_t s);

// Plan-time state of prediction and calibration: device copies of uvw and the frequencies,
// and (with antennas) the per-antenna list of rows, the per-row sums and the gain buffers.
Status build_calibration(Instance &I, const double *uvw_dev, const double *freq_dev, const int32_t *a1_dev,
                         const int32_t *a2_dev, hipStream_t s) {
    void *p;
    MWG_TRY(I.arena.alloc(&p, sizeof(double) * 3 * (size_t)std::max<int64_t>(I.nrow, 1)));
    I.uvw_d = (double *)p;
    if (I.nrow > 0)
        MWG_HIP(hipMemcpyAsync(I.uvw_d, uvw_dev, sizeof(double) * 3 * (size_t)I.nrow, hipMemcpyDeviceToDevice, s));
    {
        // turns per metre of every channel, f / c, formed on the host in FP64
        std::vector<double> kf((size_t)I.nchan);
        MWG_HIP(hipMemcpyAsync(kf.data(), freq_dev, sizeof(double) * (size_t)I.nchan, hipMemcpyDeviceToHost, s));
        MWG_HIP(hipStreamSynchronize(s));
        for (double &f : kf) f = f / kC;
        MWG_TRY(I.arena.alloc(&p, sizeof(double) * (size_t)I.nchan));
        I.kf_d = (double *)p;
        MWG_HIP(hipMemcpyAsync(I.kf_d, kf.data(), sizeof(double) * (size_t)I.nchan, hipMemcpyHostToDevice, s));
        MWG_HIP(hipStreamSynchronize(s));
    }
    if (!I.has_ants) return Status::Ok();
    std::vector<int32_t> h1((size_t)I.nrow), h2((size_t)I.nrow);
    if (I.nrow > 0) {
        MWG_HIP(hipMemcpyAsync(h1.data(), a1_dev, 4 * (size_t)I.nrow, hipMemcpyDeviceToHost, s));
        MWG_HIP(hipMemcpyAsync(h2.data(), a2_dev, 4 * (size_t)I.nrow, hipMemcpyDeviceToHost, s));
    }
    MWG_HIP(hipStreamSynchronize(s));
    // rows of each antenna: entry = row << 1 | (0: as ant1, 1: as ant2), rows ascending
    std::vector<int32_t> start((size_t)I.nant + 1, 0), entry(2 * (size_t)I.nrow), partner(2 * (size_t)I.nrow);
    for (int64_t r = 0; r < I.nrow; r++) {
        start[h1[r] + 1]++;
        start[h2[r] + 1]++;
    }
    for (int a = 0; a < I.nant; a++) start[a + 1] += start[a];
    {
        std::vector<int32_t> fill(start.begin(), start.end() - 1);
        for (int64_t r = 0; r < I.nrow; r++) {
            partner[fill[h1[r]]] = h2[r];
            entry[fill[h1[r]]++] = (int32_t)(r << 1);
            partner[fill[h2[r]]] = h1[r];
            entry[fill[h2[r]]++] = (int32_t)(r << 1 | 1);
        }
    }
    if (I.nrow >= (int64_t)1 << 30) return make_error(MW_ERR_UNSUPPORTED, "calibration lists need nrow < 2^30");
    MWG_TRY(I.arena.alloc(&p, 4 * start.size()));
    I.cal_start = (int32_t *)p;
    MWG_TRY(I.arena.alloc(&p, 4 * std::max<size_t>(entry.size(), 1)));
    I.cal_entry = (int32_t *)p;
    MWG_TRY(I.arena.alloc(&p, 4 * std::max<size_t>(partner.size(), 1)));
    I.cal_partner = (int32_t *)p;
    MWG_TRY(I.arena.alloc(&p, sizeof(float4) * (size_t)std::max<int64_t>(I.nrow, 1)));
    I.cal_pq = (float4 *)p;
    MWG_TRY(I.arena.alloc(&p, sizeof(float2) * (size_t)I.nant));
    I.cal_g = (float2 *)p;
    MWG_TRY(I.arena.alloc(&p, sizeof(double) * 2 * (size_t)I.nant));
    I.cal_red = (double *)p;
    MWG_HIP(hipMemcpyAsync(I.cal_start, start.data(), 4 * start.size(), hipMemcpyHostToDevice, s));
    if (!entry.empty()) {
        MWG_HIP(hipMemcpyAsync(I.cal_entry, entry.data(), 4 * entry.size(), hipMemcpyHostToDevice, s));
        MWG_HIP(hipMemcpyAsync(I.cal_partner, partner.data(), 4 * partner.size(), hipMemcpyHostToDevice, s));
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
    hipLaunchKernelGGL(k_predict, dim3(grid1d(I.ngroups)), dim3(kBlock), 0, s, I.uvw_d, I.kf_d, I.ngroups, I.nchan,
                       I.npol, (const Src *)I.src_d, nsrc, gains, I.ant_orig, out, accumulate);
    MWG_HIP(hipGetLastError());
    return Status::Ok();
}

Status launch_solve_gains(Instance &I, const float2 *vis, const float2 *model, const float *weights, float2 *gains,
                          int niter, float *rel, hipStream_t s) {
    if (!I.has_ants) return make_error(MW_ERR_STATE, "gain solving needs an instance planned with antennas");
    if (niter < 0) return make_error(MW_ERR_INVALID_ARG, "niter must be >= 0");
    return solve(I, vis, model, nullptr, weights, gains, niter, rel, s);
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
    for (int k : order) {
        float2 *gk = gains + (size_t)k * I.nant;
        hipLaunchKernelGGL(k_fill_gains, dim3(grid1d(I.nant)), dim3(kBlock), 0, s, gk, I.nant, make_float2(1.f, 0.f));
        MWG_HIP(hipGetLastError());
        MWG_TRY(solve(I, resid, nullptr, table + k, weights, gk, niter, rel ? rel + k : nullptr, s));
        hipLaunchKernelGGL(k_predict, dim3(grid1d(I.ngroups)), dim3(kBlock), 0, s, I.uvw_d, I.kf_d, I.ngroups,
                           I.nchan, I.npol, table + nsrc + k, 1, (const float2 *)gk, I.ant_orig, resid, 1);
        MWG_HIP(hipGetLastError());
    }
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
