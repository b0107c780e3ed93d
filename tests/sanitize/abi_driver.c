/* The C ABI's argument checking under AddressSanitizer and UndefinedBehaviorSanitizer (the
 * library's host code built with both): every entry point is called with missing, dead and
 * out-of-range arguments and must return its documented status with a message, touching no
 * GPU. Exits non-zero on a wrong status. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "mwagrid.h"

static int expect(mw_status got, mw_status want, const char *what) {
    if (got != want) {
        fprintf(stderr, "%s: status %d, expected %d (%s)\n", what, (int)got, (int)want, mw_last_error());
        return 1;
    }
    if (want != MW_OK && strlen(mw_last_error()) == 0) {
        fprintf(stderr, "%s: no message\n", what);
        return 1;
    }
    return 0;
}

int main(void) {
    int bad = 0;
    double uvw[12] = {0}, freq[1] = {150e6};
    mw_instance d;
    memset(&d, 0, sizeof d);
    d.nx = d.ny = 64;
    d.du = d.dv = 1.0;
    d.nrow = 4;
    d.nchan = 1;
    d.npol = 1;
    d.uvw_m = uvw;
    d.freq_hz = freq;
    d.support = 7;
    d.oversample = 8;
    d.mem = MW_MEM_HOST;
    mw_plan h = NULL;
    struct {
        const char *what;
        void (*set)(mw_instance *);
    } cases[1];
    (void)cases;
    mw_instance e;
#define CASE(stmt, code)                                                                         \
    do {                                                                                         \
        e = d;                                                                                   \
        stmt;                                                                                    \
        bad |= expect(mw_grid_plan(&h, &e, 1, NULL, NULL), code, #stmt);                         \
        bad |= h != NULL;                                                                        \
    } while (0)
    CASE(e.nx = 63, MW_ERR_INVALID_ARG);
    CASE(e.nx = 8192, MW_ERR_UNSUPPORTED);
    CASE(e.du = NAN, MW_ERR_INVALID_ARG);
    CASE(e.npol = 3, MW_ERR_INVALID_ARG);
    CASE(e.support = 8, MW_ERR_INVALID_ARG);
    CASE(e.oversample = 17, MW_ERR_INVALID_ARG);
    CASE(e.uvw_m = NULL, MW_ERR_INVALID_ARG);
    CASE(e.weighting = 3, MW_ERR_INVALID_ARG);
    CASE(e.robust = INFINITY, MW_ERR_INVALID_ARG);
    CASE((e.wlo = 2.0, e.whi = 1.0), MW_ERR_INVALID_ARG);
    CASE(e.nrow = (int64_t)1 << 30; e.nchan = 4, MW_ERR_UNSUPPORTED);
    mw_tuning t;
    memset(&t, 0, sizeof t);
    t.flush = 4;
    bad |= expect(mw_grid_plan(&h, &d, 1, &t, NULL), MW_ERR_INVALID_ARG, "flush 4");
    bad |= expect(mw_grid_plan(NULL, &d, 1, NULL, NULL), MW_ERR_INVALID_ARG, "null out");
    bad |= expect(mw_grid_plan(&h, NULL, 1, NULL, NULL), MW_ERR_INVALID_ARG, "null inst");
    mw_plan dead = (mw_plan)(void *)0x1000;
    bad |= expect(mw_grid(NULL, NULL, NULL, NULL, 0, NULL), MW_ERR_INVALID_ARG, "grid null");
    bad |= expect(mw_grid(dead, NULL, NULL, NULL, 0, NULL), MW_ERR_STATE, "grid dead");
    bad |= expect(mw_grid_noalloc(dead, NULL, NULL, NULL, 0, NULL), MW_ERR_STATE, "noalloc dead");
    bad |= expect(mw_degrid(NULL, NULL, NULL, NULL, NULL, NULL, NULL), MW_ERR_INVALID_ARG, "degrid null");
    bad |= expect(mw_image(dead, NULL, NULL, 1, 0, NULL), MW_ERR_STATE, "image dead");
    bad |= expect(mw_stokes(NULL, NULL, NULL, NULL, NULL), MW_ERR_INVALID_ARG, "stokes null");
    bad |= expect(mw_predict(dead, 0, NULL, 0, NULL, NULL, 0, NULL), MW_ERR_STATE, "predict dead");
    bad |= expect(mw_solve_gains(NULL, 0, NULL, NULL, NULL, NULL, 1, NULL, NULL), MW_ERR_INVALID_ARG, "solve null");
    bad |= expect(mw_peel(dead, 0, NULL, NULL, 0, NULL, 1, NULL, NULL, NULL, NULL), MW_ERR_STATE, "peel dead");
    bad |= expect(mw_wstack_combine(dead, NULL, NULL, 0, NULL), MW_ERR_STATE, "wstack dead");
    mw_plan_stats st;
    bad |= expect(mw_plan_info(dead, 0, &st), MW_ERR_STATE, "info dead");
    bad |= expect(mw_plan_destroy(dead), MW_ERR_STATE, "destroy dead");
    bad |= expect(mw_plan_destroy(NULL), MW_OK, "destroy null");
    bad |= mw_abi_version() != MW_ABI_VERSION;
    if (!bad) printf("abi checks passed\n");
    return bad;
}
