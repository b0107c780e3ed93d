// Prolate spheroidal kernel tables for the gridder and the image correction.
//
// The paper fixes no gridding kernel (Section 2.1 says only that a convolution interpolates
// the visibilities onto a regular grid; Table 1 lists a "Convolution Correction" step). This
// library uses the zeroth prolate spheroidal wave function psi_0(c, eta) with c = pi*W/2:
// the kernel is C(t) = psi_0(c, 2t/W) on |t| <= W/2, and the correction is its normalised
// Fourier transform, which by the finite-Fourier-transform eigen-property equals
// psi_0(c, 2x)/psi_0(c, 0).
//
// psi_0 is even, so in orthonormal Legendre polynomials only even degrees k = 2j occur, and
// the prolate operator -d/deta (1 - eta^2) d/deta + c^2 eta^2 restricted to them is the
// symmetric tridiagonal matrix
//   diag_j = k(k+1) + c^2 (a_k^2 + a_{k+1}^2),  off_j = c^2 a_{k+1} a_{k+2},
//   a_k = k / sqrt((2k-1)(2k+1)),
// (a_k are the off-diagonal entries of multiplication by eta). Its smallest eigenvalue is
// found by Sturm-sequence bisection and the eigenvector by inverse iteration.
#include "internal.h"

#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

namespace mwg {

namespace {

struct Prolate {
    std::vector<double> coef;    // coefficient of P_{2j} (standard Legendre)
    std::vector<double> ra, rb;  // recurrence factors (2k+1)/(k+1) and k/(k+1)
};

double legendre_a(int k) { return k == 0 ? 0.0 : k / std::sqrt((2.0 * k - 1.0) * (2.0 * k + 1.0)); }

// Number of eigenvalues of the tridiagonal (d, e) strictly below x.
int sturm_count(const std::vector<double> &d, const std::vector<double> &e, double x) {
    int n = (int)d.size(), count = 0;
    double q = d[0] - x;
    if (q < 0) count++;
    for (int i = 1; i < n; i++) {
        double qq = (q == 0.0) ? 1e-300 : q;
        q = (d[i] - x) - e[i - 1] * e[i - 1] / qq;
        if (q < 0) count++;
    }
    return count;
}

Prolate solve(double c) {
    const int m = (int)std::ceil(c) + 40; // even-degree terms; coefficients decay super-exponentially
    std::vector<double> d(m), e(m - 1);
    for (int j = 0; j < m; j++) {
        int k = 2 * j;
        double ak = legendre_a(k), ak1 = legendre_a(k + 1);
        d[j] = k * (k + 1.0) + c * c * (ak * ak + ak1 * ak1);
        if (j + 1 < m) e[j] = c * c * legendre_a(k + 1) * legendre_a(k + 2);
    }
    // Gershgorin interval, then bisection for the smallest eigenvalue.
    double lo = d[0], hi = d[0];
    for (int j = 0; j < m; j++) {
        double r = (j > 0 ? std::fabs(e[j - 1]) : 0.0) + (j + 1 < m ? std::fabs(e[j]) : 0.0);
        lo = std::fmin(lo, d[j] - r);
        hi = std::fmax(hi, d[j] + r);
    }
    for (int it = 0; it < 200 && hi - lo > 1e-15 * std::fmax(1.0, std::fabs(hi)); it++) {
        double mid = 0.5 * (lo + hi);
        if (sturm_count(d, e, mid) >= 1) hi = mid; else lo = mid;
    }
    const double lam = 0.5 * (lo + hi);
    // Inverse iteration: solve (T - lam I) y = x with a tridiagonal LU (no pivoting needed
    // for this diagonally dominated shifted system in practice; a tiny shift guards zeros).
    std::vector<double> x(m, 1.0), y(m), cp(m), dp(m);
    for (int iter = 0; iter < 4; iter++) {
        const double shift = lam - 1e-12 * std::fmax(1.0, std::fabs(lam));
        double b0 = d[0] - shift;
        cp[0] = (m > 1 ? e[0] : 0.0) / b0;
        dp[0] = x[0] / b0;
        for (int j = 1; j < m; j++) {
            double b = (d[j] - shift) - e[j - 1] * cp[j - 1];
            cp[j] = (j + 1 < m ? e[j] : 0.0) / b;
            dp[j] = (x[j] - e[j - 1] * dp[j - 1]) / b;
        }
        y[m - 1] = dp[m - 1];
        for (int j = m - 2; j >= 0; j--) y[j] = dp[j] - cp[j] * y[j + 1];
        double nrm = 0.0;
        for (int j = 0; j < m; j++) nrm += y[j] * y[j];
        nrm = std::sqrt(nrm);
        for (int j = 0; j < m; j++) x[j] = y[j] / nrm;
    }
    Prolate p;
    p.coef.resize(m);
    for (int j = 0; j < m; j++) p.coef[j] = x[j] * std::sqrt((4.0 * j + 1.0) / 2.0);
    // sign: psi_0(0) > 0; P_{2j}(0) = (-1)^j (2j-1)!!/(2j)!!
    double at0 = 0.0, pj = 1.0;
    for (int j = 0; j < m; j++) {
        at0 += p.coef[j] * pj;
        pj *= -(2.0 * j + 1.0) / (2.0 * j + 2.0);
    }
    if (at0 < 0)
        for (double &v : p.coef) v = -v;
    p.ra.resize(2 * m);
    p.rb.resize(2 * m);
    for (int k = 0; k < 2 * m; k++) {
        p.ra[k] = (2.0 * k + 1.0) / (k + 1.0);
        p.rb[k] = k / (k + 1.0);
    }
    return p;
}

double evaluate(const Prolate &p, double eta) {
    // Bonnet recurrence: (k+1) P_{k+1} = (2k+1) eta P_k - k P_{k-1}; sum the even terms.
    double pm1 = 1.0, pk = eta, sum = p.coef[0];
    const int kmax = 2 * (int)p.coef.size() - 2;
    for (int k = 1; k < kmax; k++) {
        double pk1 = (p.ra[k] * eta * pk - p.rb[k] * pm1);
        pm1 = pk;
        pk = pk1;
        if ((k + 1) % 2 == 0) sum += p.coef[(k + 1) / 2] * pk;
    }
    return sum;
}

} // namespace

// Tables depend only on (W, O, nx, ny) and plans of many instances repeat a few of them, so
// they are computed once per process and kept (a few KiB each).
struct TableKey {
    int W, O, nx, ny;
    bool operator<(const TableKey &o) const {
        return std::tie(W, O, nx, ny) < std::tie(o.W, o.O, o.nx, o.ny);
    }
};
struct TableEntry {
    std::vector<float> table, corr_x, corr_y;
};

void prolate_tables(int W, int O, int nx, int ny, std::vector<float> &table,
                    std::vector<float> &corr_x, std::vector<float> &corr_y) {
    static std::mutex mu;
    static std::map<TableKey, TableEntry> cache;
    const TableKey key{W, O, nx, ny};
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) {
            table = it->second.table;
            corr_x = it->second.corr_x;
            corr_y = it->second.corr_y;
            return;
        }
    }
    const double c = M_PI * W / 2.0;
    Prolate p = solve(c);
    const int h = (W - 1) / 2;
    table.assign((size_t)O * W, 0.0f);
    for (int row = 0; row < O; row++) {
        const int ph = row - O / 2;
        double vals[64], sum = 0.0;
        for (int t = -h; t <= h; t++) {
            double eta = 2.0 * (t - (double)ph / O) / W;
            double v = std::fabs(eta) <= 1.0 ? evaluate(p, eta) : 0.0;
            vals[t + h] = v;
            sum += v;
        }
        for (int t = 0; t < W; t++) table[(size_t)row * W + t] = (float)(vals[t] / sum);
    }
    const double at0 = evaluate(p, 0.0);
    // psi_0 is even: pixel n/2 + d and n/2 - d take the same value, so each is evaluated once
    auto fill = [&](int n, std::vector<float> &out) {
        out.resize(n);
        for (int i = 0; i < n; i++) {
            const int mirror = n - i;  // (mirror - n/2) = -(i - n/2) when n is even
            if (n % 2 == 0 && i > n / 2 && mirror >= 0 && mirror < i) {
                out[i] = out[mirror];
                continue;
            }
            double x = (i - n / 2.0) / n;
            out[i] = (float)(evaluate(p, 2.0 * x) / at0);
        }
    };
    fill(nx, corr_x);
    fill(ny, corr_y);
    std::lock_guard<std::mutex> lk(mu);
    cache.emplace(key, TableEntry{table, corr_x, corr_y});
}

} // namespace mwg
