/* The oracle's C loops under AddressSanitizer and UndefinedBehaviorSanitizer: positions
 * (with flags, zero weights, non-finite coordinates and out-of-grid footprints), gridding and
 * degridding with weights and gains, on one and on several threads. Exits non-zero on a
 * wrong result; the sanitizers abort on any error. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void orc_positions(int64_t nrow, int32_t nchan, const double *uvw, const double *freq, const uint8_t *flags,
                   const double *weights, int32_t nx, int32_t ny, double du, double dv, int32_t O,
                   const int32_t *half, int32_t h_uniform, int32_t *pos, uint8_t *keep, int64_t *counts);
void orc_grid(int64_t ngroups, int32_t npol, const int32_t *pos, const uint8_t *keep, const double *vis,
              const double *weights, const double *gains, const int32_t *ant1, const int32_t *ant2, int32_t nchan,
              int32_t nx, int32_t ny, int32_t W, int32_t O, const double *table, double *grid, int32_t nthreads);
void orc_degrid(int64_t ngroups, int32_t npol, const int32_t *pos, const uint8_t *keep, const double *grid,
                const double *weights, const double *gains, const int32_t *ant1, const int32_t *ant2, int32_t nchan,
                int32_t nx, int32_t ny, int32_t W, int32_t O, const double *table, double *out, int32_t nthreads);

int main(void) {
    enum { NROW = 200, NCHAN = 3, NPOL = 2, NX = 64, NY = 48, W = 7, O = 8, NANT = 20 };
    const int64_t ng = (int64_t)NROW * NCHAN;
    double *uvw = malloc(sizeof(double) * 3 * NROW), freq[NCHAN] = {299792458.0, 1.1 * 299792458.0, 1.3 * 299792458.0};
    uint8_t *flags = calloc(ng, 1), *keep = malloc(ng);
    double *w = malloc(sizeof(double) * ng), *vis = malloc(sizeof(double) * 2 * NPOL * ng);
    double *gains = malloc(sizeof(double) * 2 * NANT), table[O * W];
    int32_t *pos = malloc(sizeof(int32_t) * 4 * ng), a1[NROW], a2[NROW];
    int64_t counts[3];
    srand(7);
    for (int r = 0; r < NROW; r++) {
        uvw[3 * r] = (rand() / (double)RAND_MAX - 0.5) * 70.0;
        uvw[3 * r + 1] = (rand() / (double)RAND_MAX - 0.5) * 50.0;
        uvw[3 * r + 2] = 0.0;
        a1[r] = r % NANT;
        a2[r] = (r * 7 + 3) % NANT;
    }
    uvw[0] = NAN;
    uvw[4] = INFINITY;
    uvw[6] = 1e300;
    for (int64_t g = 0; g < ng; g++) {
        flags[g] = (g % 17) == 0;
        w[g] = (g % 23) == 0 ? 0.0 : 0.5 + (double)(g % 5) / 4.0;
    }
    for (int64_t i = 0; i < 2 * NPOL * ng; i++) vis[i] = rand() / (double)RAND_MAX - 0.5;
    for (int a = 0; a < NANT; a++) {
        gains[2 * a] = 1.0 + 0.01 * a;
        gains[2 * a + 1] = -0.02 * a;
    }
    for (int p = 0; p < O; p++)
        for (int t = 0; t < W; t++) table[p * W + t] = 1.0 / W;
    orc_positions(NROW, NCHAN, uvw, freq, flags, w, NX, NY, 1.0, 1.0, O, NULL, (W - 1) / 2, pos, keep, counts);
    if (counts[0] + counts[1] + counts[2] != ng || counts[0] == 0 || counts[2] == 0) return 3;
    double *g1 = calloc(2 * NPOL * NX * NY, sizeof(double)), *g4 = calloc(2 * NPOL * NX * NY, sizeof(double));
    orc_grid(ng, NPOL, pos, keep, vis, w, gains, a1, a2, NCHAN, NX, NY, W, O, table, g1, 1);
    orc_grid(ng, NPOL, pos, keep, vis, w, gains, a1, a2, NCHAN, NX, NY, W, O, table, g4, 4);
    if (memcmp(g1, g4, sizeof(double) * 2 * NPOL * NX * NY) != 0) return 4; /* bit-identical threads */
    double *o1 = calloc(2 * NPOL * ng, sizeof(double)), *o4 = calloc(2 * NPOL * ng, sizeof(double));
    orc_degrid(ng, NPOL, pos, keep, g1, w, gains, a1, a2, NCHAN, NX, NY, W, O, table, o1, 1);
    orc_degrid(ng, NPOL, pos, keep, g1, w, gains, a1, a2, NCHAN, NX, NY, W, O, table, o4, 3);
    if (memcmp(o1, o4, sizeof(double) * 2 * NPOL * ng) != 0) return 5;
    free(uvw); free(flags); free(keep); free(w); free(vis); free(gains); free(pos);
    free(g1); free(g4); free(o1); free(o4);
    printf("oracle checks passed\n");
    return 0;
}
