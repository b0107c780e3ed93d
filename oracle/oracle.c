/*
 * Oracle for convolutional gridding and its adjoint: plain loops in FP64.
 *
 * Test infrastructure only. Nothing in the product library links or calls this file;
 * only tests/, __graft_entry__.smoke() and the cpu_baseline leg of bench.py use it, through
 * oracle/__init__.py. It shares no code or headers with the HIP path. Build flags:
 * -O2 -ffp-contract=off (every operation rounded to FP64 in the written order).
 *
 * What is computed follows the paper's one-sentence statement of the step (Section 2.1:
 * the visibilities are convolved so that they are interpolated onto a regular grid, which
 * the FFT then turns into images), with the readings that make it concrete:
 *   positions   u = (u_m * f) / c_light,  x = u/du + nx/2        (grid origin at nx/2)
 *   quantise    qx = floor(x*O + 1/2); cx = floor((qx + O/2)/O); px = qx - cx*O
 *   keep        not flagged, weight != 0, and cx-h >= 0, cx+h < nx (same for y)
 *   grid        G[pol][cy+s][cx+t] += w * g1 * conj(g2) * T[py][s] * T[px][t] * V[pol]
 *   degrid      y[pol] = w * conj(g1) * g2 * sum_{s,t} T[py][s] * T[px][t] * G[pol][cy+s][cx+t]
 * and the kernel-stack form, in which a complex tap K[py][px][s][t] selected per visibility
 * replaces the separable product (conjugated in the adjoint).
 *
 * Multi-threaded gridding gives each thread a stripe of grid rows; every thread visits the
 * visibilities in ascending order, so each cell receives its terms in the same order as the
 * single-threaded loop and the result is bit-identical for any thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_C_LIGHT 299792458.0

static int64_t orc_floor_div(int64_t a, int64_t b)
{
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0)))
        q -= 1;
    return q;
}

/*
 * Positions, quantisation and the keep rule for every (row, channel) group.
 * half: per-group half support (kernel stacks) or NULL to use h_uniform.
 * pos:  [ngroups][4] = cx, cy, px, py; all -1 for a dropped group.
 * keep: [ngroups] 1 if gridded.
 * counts: [3] = kept, flagged (flag set or zero weight), outside (footprint leaves grid or
 *         non-finite position).
 */
void orc_positions(int64_t nrow, int32_t nchan, const double *uvw, const double *freq,
                   const uint8_t *flags, const double *weights, int32_t nx, int32_t ny,
                   double du, double dv, int32_t O, const int32_t *half, int32_t h_uniform,
                   int32_t *pos, uint8_t *keep, int64_t *counts)
{
    int64_t nkept = 0, nflag = 0, nout = 0;
    for (int64_t r = 0; r < nrow; r++) {
        for (int32_t ch = 0; ch < nchan; ch++) {
            int64_t g = r * nchan + ch;
            int32_t *pg = pos + 4 * g;
            pg[0] = pg[1] = pg[2] = pg[3] = -1;
            keep[g] = 0;
            if ((flags && flags[g]) || (weights && weights[g] == 0.0)) {
                nflag++;
                continue;
            }
            double f = freq[ch];
            double u = (uvw[3 * r + 0] * f) / ORC_C_LIGHT;
            double v = (uvw[3 * r + 1] * f) / ORC_C_LIGHT;
            double x = u / du + (double)(nx / 2);
            double y = v / dv + (double)(ny / 2);
            double qxd = floor(x * (double)O + 0.5);
            double qyd = floor(y * (double)O + 0.5);
            if (!(fabs(qxd) < 1e15) || !(fabs(qyd) < 1e15)) {
                nout++;
                continue;
            }
            int64_t qx = (int64_t)qxd, qy = (int64_t)qyd;
            int64_t cx = orc_floor_div(qx + O / 2, O);
            int64_t cy = orc_floor_div(qy + O / 2, O);
            int64_t px = qx - cx * O;
            int64_t py = qy - cy * O;
            int64_t h = half ? half[g] : h_uniform;
            if (cx - h < 0 || cx + h >= nx || cy - h < 0 || cy + h >= ny) {
                nout++;
                continue;
            }
            pg[0] = (int32_t)cx;
            pg[1] = (int32_t)cy;
            pg[2] = (int32_t)px;
            pg[3] = (int32_t)py;
            keep[g] = 1;
            nkept++;
        }
    }
    counts[0] = nkept;
    counts[1] = nflag;
    counts[2] = nout;
}

/* Complex multiplier w * g1 * conj(g2) (forward) for group g; 1 when both are absent. */
static void orc_multiplier(int64_t g, int32_t nchan, const double *weights, const double *gains,
                           const int32_t *ant1, const int32_t *ant2, int conj_form,
                           double *mr, double *mi)
{
    double ar = 1.0, ai = 0.0;
    if (gains) {
        int64_t row = g / nchan;
        const double *g1 = gains + 2 * (int64_t)ant1[row];
        const double *g2 = gains + 2 * (int64_t)ant2[row];
        if (!conj_form) { /* g1 * conj(g2) */
            ar = g1[0] * g2[0] + g1[1] * g2[1];
            ai = g1[1] * g2[0] - g1[0] * g2[1];
        } else { /* conj(g1) * g2 */
            ar = g1[0] * g2[0] + g1[1] * g2[1];
            ai = g1[0] * g2[1] - g1[1] * g2[0];
        }
    }
    double w = weights ? weights[g] : 1.0;
    *mr = w * ar;
    *mi = w * ai;
}

/*
 * Separable-kernel gridding, accumulated into grid [npol][ny][nx][2].
 * vis [ngroups][npol][2]; table [O][W] (row = phase + O/2, column = tap + h).
 */
void orc_grid(int64_t ngroups, int32_t npol, const int32_t *pos, const uint8_t *keep,
              const double *vis, const double *weights, const double *gains,
              const int32_t *ant1, const int32_t *ant2, int32_t nchan, int32_t nx, int32_t ny,
              int32_t W, int32_t O, const double *table, double *grid, int32_t nthreads)
{
    const int32_t h = (W - 1) / 2;
    if (nthreads < 1)
        nthreads = 1;
#pragma omp parallel num_threads(nthreads)
    {
        int32_t tid = 0, nth = 1;
#ifdef _OPENMP
        tid = omp_get_thread_num();
        nth = omp_get_num_threads();
#endif
        int32_t y0 = (int32_t)(((int64_t)ny * tid) / nth);
        int32_t y1 = (int32_t)(((int64_t)ny * (tid + 1)) / nth);
        double zr[16], zi[16];
        for (int64_t g = 0; g < ngroups; g++) {
            if (!keep[g])
                continue;
            const int32_t *pg = pos + 4 * g;
            int32_t cx = pg[0], cy = pg[1], px = pg[2], py = pg[3];
            if (cy + h < y0 || cy - h >= y1)
                continue;
            double mr, mi;
            orc_multiplier(g, nchan, weights, gains, ant1, ant2, 0, &mr, &mi);
            for (int32_t p = 0; p < npol; p++) {
                double vr = vis[(g * npol + p) * 2 + 0];
                double vi = vis[(g * npol + p) * 2 + 1];
                zr[p] = mr * vr - mi * vi;
                zi[p] = mr * vi + mi * vr;
            }
            const double *ty = table + (int64_t)(py + O / 2) * W;
            const double *tx = table + (int64_t)(px + O / 2) * W;
            for (int32_t s = -h; s <= h; s++) {
                int32_t y = cy + s;
                if (y < y0 || y >= y1)
                    continue;
                for (int32_t t = -h; t <= h; t++) {
                    int32_t x = cx + t;
                    double tap = ty[s + h] * tx[t + h];
                    for (int32_t p = 0; p < npol; p++) {
                        double *cell = grid + (((int64_t)p * ny + y) * nx + x) * 2;
                        cell[0] += tap * zr[p];
                        cell[1] += tap * zi[p];
                    }
                }
            }
        }
    }
}

/*
 * Separable-kernel degridding (adjoint of orc_grid without the accumulation):
 * out [ngroups][npol][2] = w * conj(g1) * g2 * sum_{s,t} tap * grid; zero for dropped groups.
 */
void orc_degrid(int64_t ngroups, int32_t npol, const int32_t *pos, const uint8_t *keep,
                const double *grid, const double *weights, const double *gains,
                const int32_t *ant1, const int32_t *ant2, int32_t nchan, int32_t nx, int32_t ny,
                int32_t W, int32_t O, const double *table, double *out, int32_t nthreads)
{
    const int32_t h = (W - 1) / 2;
    if (nthreads < 1)
        nthreads = 1;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t g = 0; g < ngroups; g++) {
        double ar[16], ai[16];
        for (int32_t p = 0; p < npol; p++)
            ar[p] = ai[p] = 0.0;
        if (keep[g]) {
            const int32_t *pg = pos + 4 * g;
            int32_t cx = pg[0], cy = pg[1], px = pg[2], py = pg[3];
            const double *ty = table + (int64_t)(py + O / 2) * W;
            const double *tx = table + (int64_t)(px + O / 2) * W;
            for (int32_t s = -h; s <= h; s++) {
                for (int32_t t = -h; t <= h; t++) {
                    double tap = ty[s + h] * tx[t + h];
                    for (int32_t p = 0; p < npol; p++) {
                        const double *cell =
                            grid + (((int64_t)p * ny + (cy + s)) * nx + (cx + t)) * 2;
                        ar[p] += tap * cell[0];
                        ai[p] += tap * cell[1];
                    }
                }
            }
            double mr, mi;
            orc_multiplier(g, nchan, weights, gains, ant1, ant2, 1, &mr, &mi);
            for (int32_t p = 0; p < npol; p++) {
                double r = mr * ar[p] - mi * ai[p];
                double i = mr * ai[p] + mi * ar[p];
                ar[p] = r;
                ai[p] = i;
            }
        }
        for (int32_t p = 0; p < npol; p++) {
            out[(g * npol + p) * 2 + 0] = ar[p];
            out[(g * npol + p) * 2 + 1] = ai[p];
        }
    }
}

/*
 * Kernel-stack gridding. Kernel k has odd support S = ksupport[k] and its complex taps sit
 * at kstack + 2*koffset[k] as [O][O][S][S][2] (phase row py+O/2, phase column px+O/2, tap
 * row s+h, tap column t+h). kidx [ngroups] selects the kernel of each group.
 */
void orc_grid_stack(int64_t ngroups, int32_t npol, const int32_t *pos, const uint8_t *keep,
                    const double *vis, const double *weights, const double *gains,
                    const int32_t *ant1, const int32_t *ant2, int32_t nchan, int32_t nx,
                    int32_t ny, int32_t O, const double *kstack, const int64_t *koffset,
                    const int32_t *ksupport, const int32_t *kidx, double *grid, int32_t nthreads)
{
    if (nthreads < 1)
        nthreads = 1;
#pragma omp parallel num_threads(nthreads)
    {
        int32_t tid = 0, nth = 1;
#ifdef _OPENMP
        tid = omp_get_thread_num();
        nth = omp_get_num_threads();
#endif
        int32_t y0 = (int32_t)(((int64_t)ny * tid) / nth);
        int32_t y1 = (int32_t)(((int64_t)ny * (tid + 1)) / nth);
        double zr[16], zi[16];
        for (int64_t g = 0; g < ngroups; g++) {
            if (!keep[g])
                continue;
            const int32_t *pg = pos + 4 * g;
            int32_t cx = pg[0], cy = pg[1], px = pg[2], py = pg[3];
            int32_t k = kidx[g];
            int32_t S = ksupport[k];
            int32_t h = (S - 1) / 2;
            if (cy + h < y0 || cy - h >= y1)
                continue;
            double mr, mi;
            orc_multiplier(g, nchan, weights, gains, ant1, ant2, 0, &mr, &mi);
            for (int32_t p = 0; p < npol; p++) {
                double vr = vis[(g * npol + p) * 2 + 0];
                double vi = vis[(g * npol + p) * 2 + 1];
                zr[p] = mr * vr - mi * vi;
                zi[p] = mr * vi + mi * vr;
            }
            const double *kt = kstack + 2 * (koffset[k] +
                                             ((int64_t)(py + O / 2) * O + (px + O / 2)) * S * S);
            for (int32_t s = -h; s <= h; s++) {
                int32_t y = cy + s;
                if (y < y0 || y >= y1)
                    continue;
                for (int32_t t = -h; t <= h; t++) {
                    int32_t x = cx + t;
                    double kr = kt[((int64_t)(s + h) * S + (t + h)) * 2 + 0];
                    double ki = kt[((int64_t)(s + h) * S + (t + h)) * 2 + 1];
                    for (int32_t p = 0; p < npol; p++) {
                        double *cell = grid + (((int64_t)p * ny + y) * nx + x) * 2;
                        cell[0] += kr * zr[p] - ki * zi[p];
                        cell[1] += kr * zi[p] + ki * zr[p];
                    }
                }
            }
        }
    }
}

/* Kernel-stack degridding: conjugated taps; otherwise as orc_degrid. */
void orc_degrid_stack(int64_t ngroups, int32_t npol, const int32_t *pos, const uint8_t *keep,
                      const double *grid, const double *weights, const double *gains,
                      const int32_t *ant1, const int32_t *ant2, int32_t nchan, int32_t nx,
                      int32_t ny, int32_t O, const double *kstack, const int64_t *koffset,
                      const int32_t *ksupport, const int32_t *kidx, double *out,
                      int32_t nthreads)
{
    if (nthreads < 1)
        nthreads = 1;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t g = 0; g < ngroups; g++) {
        double ar[16], ai[16];
        for (int32_t p = 0; p < npol; p++)
            ar[p] = ai[p] = 0.0;
        if (keep[g]) {
            const int32_t *pg = pos + 4 * g;
            int32_t cx = pg[0], cy = pg[1], px = pg[2], py = pg[3];
            int32_t k = kidx[g];
            int32_t S = ksupport[k];
            int32_t h = (S - 1) / 2;
            const double *kt = kstack + 2 * (koffset[k] +
                                             ((int64_t)(py + O / 2) * O + (px + O / 2)) * S * S);
            for (int32_t s = -h; s <= h; s++) {
                for (int32_t t = -h; t <= h; t++) {
                    double kr = kt[((int64_t)(s + h) * S + (t + h)) * 2 + 0];
                    double ki = -kt[((int64_t)(s + h) * S + (t + h)) * 2 + 1];
                    for (int32_t p = 0; p < npol; p++) {
                        const double *cell =
                            grid + (((int64_t)p * ny + (cy + s)) * nx + (cx + t)) * 2;
                        ar[p] += kr * cell[0] - ki * cell[1];
                        ai[p] += kr * cell[1] + ki * cell[0];
                    }
                }
            }
            double mr, mi;
            orc_multiplier(g, nchan, weights, gains, ant1, ant2, 1, &mr, &mi);
            for (int32_t p = 0; p < npol; p++) {
                double r = mr * ar[p] - mi * ai[p];
                double i = mr * ai[p] + mi * ar[p];
                ar[p] = r;
                ai[p] = i;
            }
        }
        for (int32_t p = 0; p < npol; p++) {
            out[(g * npol + p) * 2 + 0] = ar[p];
            out[(g * npol + p) * 2 + 1] = ai[p];
        }
    }
}
