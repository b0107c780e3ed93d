/*
 * mwagrid.h - C ABI of libmwagrid, convolutional gridding of radio visibilities onto the
 * uv-plane, the FFT to per-polarisation images with kernel correction, and the exact
 * adjoints of both, on one AMD Instinct MI355X (gfx950).
 *
 * The operations follow the paper's statement of the imaging step: the calibrated
 * visibilities, samples of the Fourier transform of the sky (Section 2.1), are convolved so
 * that they are interpolated onto a regular grid on which an FFT can operate (Section 2.1);
 * the FFT turns the grid into images, one per instrumental polarisation (Section 2,
 * Section 2.1), which are then convolution-corrected (Table 1: Gridding, FFT, Convolution
 * Correction). The paper fixes no kernel, grid convention or precision; the rules used here
 * are stated at each call.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - A "group" is one (row, channel) pair; a row is one baseline at one time. Group g =
 *    row * nchan + chan. Visibilities are complex64 (float re, float im) laid out
 *    [ngroups][npol], contiguous.
 *  - A grid or image is complex64 [npol][ny][nx], contiguous (x fastest). Column x holds
 *    u = (x - nx/2) * du, row y holds v = (y - ny/2) * dv.
 *  - Positions (computed once, in FP64, at plan time): u = (u_m * f) / 299792458,
 *    x = u/du + nx/2, qx = floor(x*O + 1/2), cx = floor((qx + O/2)/O), px = qx - cx*O; the
 *    same for y. A group is dropped (never gridded, adjoint output zero) if it is flagged, its
 *    weight is zero, its position is not finite, or its footprint [cx-h, cx+h] x [cy-h, cy+h]
 *    leaves the grid (h = (W-1)/2, or the half support of its kernel for stacks).
 *  - Built-in kernel: the zeroth prolate spheroidal wave function C(t) = psi_0(c, 2t/W),
 *    c = pi*W/2, tabulated at O phases; each phase row is normalised to unit sum. Tap of
 *    group g at cell (cx+t, cy+s) is T[py][s] * T[px][t].
 *  - Device pointers passed to grid/degrid/image must be on the device that was current when
 *    the plan was made; "stream" is a hipStream_t (NULL = the null stream). Those calls only
 *    enqueue work; kernel faults surface at the caller's next synchronisation.
 *  - Every call returns an mw_status; on failure mw_last_error() describes it. No call
 *    aborts, prints or throws across this boundary. A plan serves one stream at a time;
 *    concurrent calls on one plan from several threads are not supported.
 */
#ifndef MWAGRID_H
#define MWAGRID_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MW_ABI_VERSION 5

typedef enum {
    MW_OK = 0,
    MW_ERR_INVALID_ARG = 1, /* a null pointer, size or option outside its documented range */
    MW_ERR_UNSUPPORTED = 2, /* valid in principle but beyond this build's limits */
    MW_ERR_ALLOC = 3,       /* device or pinned host allocation failed */
    MW_ERR_HIP = 4,         /* a HIP runtime or rocFFT call failed */
    MW_ERR_STATE = 5        /* the plan cannot serve this call (e.g. destroyed, wrong form) */
} mw_status;

enum { MW_MEM_HOST = 0, MW_MEM_DEVICE = 1 };

typedef struct mw_plan_s *mw_plan; /* opaque; owned by the library until mw_plan_destroy */

/*
 * One gridding instance: one grid, the visibilities' coordinates and how to weight them.
 * Arrays are read during mw_grid_plan only (host or device memory as "mem" says); the plan
 * keeps its own copies of everything it needs afterwards.
 */
typedef struct {
    int32_t nx, ny;               /* grid size; even, 8 <= n <= 4096 */
    double du, dv;                /* cell size in wavelengths, > 0 */
    int64_t nrow;                 /* rows (baseline-times); ngroups = nrow * nchan < 2^31 */
    int32_t nchan;                /* channels, >= 1 */
    int32_t npol;                 /* polarisations per group: 1, 2 or 4 */
    const double *uvw_m;          /* [nrow][3] baseline coordinates in metres (w unused) */
    const double *freq_hz;        /* [nchan] channel frequencies */
    const uint8_t *flags;         /* [ngroups] nonzero = flagged; NULL = none */
    const float *weights;         /* [ngroups] real weights; NULL = all 1 */
    const int32_t *ant1, *ant2;   /* [nrow] antenna indices in [0, nant); NULL = no gains */
    int32_t nant;                 /* antennas (when ant1/ant2 are given), <= 65535 */
    int32_t support;              /* W: odd, 1 <= W <= 15 (built-in kernel; 0 with stacks) */
    int32_t oversample;           /* O: 1 <= O <= 16 */
    /* Kernel stacks (NULL kernel_stack = built-in kernel). Kernel k has odd support
     * S = kernel_support[k] (1 <= S <= 63) and complex64 taps at element
     * kernel_offset[k] of kernel_stack laid out [O][O][S][S]: phase row py + O/2, phase
     * column px + O/2, tap row s + h, tap column t + h. kernel_index[g] selects the kernel
     * of group g. The adjoint uses conjugated taps. */
    const void *kernel_stack;
    const int64_t *kernel_offset; /* [nkernel] */
    const int32_t *kernel_support;/* [nkernel] */
    int32_t nkernel;
    int64_t kernel_elems;         /* complex elements in kernel_stack */
    const int32_t *kernel_index;  /* [ngroups] */
    int32_t mem;                  /* MW_MEM_HOST or MW_MEM_DEVICE for all arrays above */
    /* Density weighting (an imaging variant; the paper grids with the data's own weights):
     * 0 = natural (the weights as given), 1 = uniform, 2 = Briggs robust with robustness
     * "robust". The density of a cell is the summed weight W(c) of the kept groups centred in
     * it; uniform: w / W(c); robust: w / (1 + W(c) f^2), f^2 = (5 * 10^-R)^2 /
     * (sum_c W(c)^2 / sum w). The resulting weights replace the given ones in every later
     * call (grid, degrid). Cell sums are exact fixed-point integers (order-independent). */
    int32_t weighting;
    float robust;
    /* w-stacking (an imaging variant; the paper treats the array as coplanar): with
     * wlo < whi the instance grids only groups with wlo <= w < whi, w = (w_m * f) / 299792458
     * in FP64 (the others count as flagged), and the plane's w is (wlo + whi) / 2 in
     * mw_wstack_combine. wlo = whi = 0: no selection. */
    double wlo, whi;
} mw_instance;

/* Optional launch choices. Zero fields mean "choose automatically". */
typedef struct {
    int32_t tile;       /* uv tile edge in cells: 8, 16, 32 or 64 (8 needs W <= 15) */
    int32_t split;      /* max groups per work item (heavy tiles are split), >= 64 */
    int32_t wg_waves;   /* wavefronts per workgroup: 4, 8 or 16 (1 and 2 with variants 4 and 6) */
    int32_t order;      /* 1 = groups sorted by cell (then row sub-position) within a tile,
                           cells row by row, 2 = input order, 3 (default) = as 1 with the
                           cells ranked line by line across the direction from the grid
                           centre to the tile (rows or columns for tiles above 16) */
    int32_t variant;    /* gridder: 1 = tap lanes, 2 = column lanes, 3 = scatter,
                           4 = column lanes with a private tile per wavefront,
                           5 = kernel stacks, gathered by output tile (chosen for stacks),
                           6 = as 4 over a work list whose (cell, py) runs are padded to
                           blocks of 4 (flush 1 or 2, schedule 1, 3 <= W <= 7) */
    int32_t flush;      /* 1 = atomic adds of each finished tile into the zeroed grid,
                           2 = tiles to a scratch buffer, then a merge pass writes the grid
                           (with variants 4 and 6 the result is then bit-reproducible),
                           3 = owner tiles (variant 4, schedule 1, tile >= W - 1): each
                           output tile is gridded by one wavefront from every group whose
                           footprint reaches it and written once, no scratch, no merge
                           (bit-reproducible; for sparse instances). A multi-instance plan
                           takes 3 by itself for instances with at most 4096 such groups
                           per output tile */
    int32_t autotune;   /* 1 = time candidate launches (tile, waves, split, schedule; the
                           default launch first) on this plan's own positions and keep the
                           fastest. Non-zero fields above stay fixed; flush stays 2 (the
                           bit-reproducible merge) unless set to 1 here. A plan of several
                           instances that can share one launch (same npol, W, O, built-in
                           kernel) is timed as a whole batched sequence, one launch for all
                           its instances, and stays batched. If the environment variable
                           MW_TUNE_CACHE names a file, results are read from and appended to
                           it, keyed by grid size, W, O, npol and the order of magnitude of
                           the visibility count (for batches: the instance count, total
                           visibilities and total cells) */
    int32_t schedule;   /* work-item order: 1 = largest first, 2 = Z-order of tiles split into
                           8 equal-work chunks, one per XCD (variant 4 only), 3 = largest
                           first, each item shared by up to wg_waves waves of one workgroup
                           (about split / wg_waves groups per wave), their tiles summed in
                           wave order (variant 4 with flush 2 only) */
} mw_tuning;

typedef struct {
    int64_t ngroups, nkept, nflagged, noutside;
    int32_t ntiles, nwork;        /* non-empty tiles and work items */
    int32_t tile, split, wg_waves, order, variant, flush; /* the launch actually chosen */
    int32_t schedule;
    int64_t plan_bytes;           /* device memory owned by the plan for this instance */
    int32_t batched;              /* 1: the plan's instances run as one batched launch
                                     sequence (replayed from a captured graph); 0: one by one */
    int32_t pad0;
} mw_plan_stats;

/*
 * Build a plan for ninst instances (ninst >= 1), the set-up of the interpolation of the
 * samples onto a regular grid (Section 2.1). Computes every group's position in FP64
 * (the quantisation rule above), drops flagged and out-of-grid groups, sorts the kept ones
 * by uv tile (and cell), splits heavy tiles into work items, builds the kernel table and
 * correction vectors, and (ninst > 1) the persistent batched schedule. Synchronous: returns
 * after all work on "stream" is done. tuning may be NULL. On success *out owns device memory
 * until mw_plan_destroy.
 * Errors: MW_ERR_INVALID_ARG (null out/inst, a field out of range), MW_ERR_UNSUPPORTED
 * (limits above), MW_ERR_ALLOC, MW_ERR_HIP.
 */
mw_status mw_grid_plan(mw_plan *out, const mw_instance *inst, int32_t ninst,
                       const mw_tuning *tuning, void *stream);

/*
 * Grid (Section 2.1: the convolution that interpolates the samples onto a regular grid for
 * the FFT; Table 1 "Gridding"): for every instance i, grid[i] (+)= sum over kept groups of
 *   w * g[ant1] * conj(g[ant2]) * tap * V[pol]   (separable or stack tap, see above).
 * vis[i]: device complex64 [ngroups][npol]. gains: NULL, or gains[i] NULL or device
 * complex64 [nant]. grid[i]: device complex64 [npol][ny][nx]. accumulate = 0 overwrites the
 * grid (zeroing is part of the call); 1 adds to it. FP32 accumulation; the summation order
 * is fixed (bit-reproducible results) only with variant 4 and flush 2 or 3, and variant 6 with flush 2.
 * Errors: MW_ERR_INVALID_ARG (null plan/arrays), MW_ERR_STATE (gains for an instance planned
 * without antennas), MW_ERR_HIP (launch failure).
 */
mw_status mw_grid(mw_plan plan, const void *const *vis, const void *const *gains,
                  void *const *grid, int32_t accumulate, void *stream);

/*
 * Grid without allocating: for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc). Computes exactly what
 * mw_grid computes, with the same kernels and summation order (identical bits), but the merge
 * flush's partial tiles live in the library's static device scratch array of 192 MiB (one per
 * GPU, held until the process ends) instead of plan-owned memory that mw_grid may allocate on
 * its first call. The call allocates nothing and frees nothing. A plan whose merge flush needs
 * more than 192 MiB of partial tiles (2 * npol * (tile + W - 1)^2 floats per work item) is
 * refused with MW_ERR_UNSUPPORTED. Instances run one after another in stream order (a batched
 * plan's graph is not used). The scratch holds no state between calls (every partial tile is
 * written before it is read), but all calls on one GPU share it: calls that overlap in time
 * on one GPU (different streams or threads) race and must be serialised by the caller.
 * Errors: as mw_grid, plus MW_ERR_UNSUPPORTED (scratch too small).
 */
mw_status mw_grid_noalloc(mw_plan plan, const void *const *vis, const void *const *gains,
                          void *const *grid, int32_t accumulate, void *stream);

/*
 * Degrid, the exact adjoint of mw_grid (the transpose of the Section 2.1 interpolation; with
 * grad_gains, the gradient with respect to the per-antenna complex gains that calibration
 * solves for, Section 2): for every instance and kept group,
 *   vis_out[g][pol] = w * conj(g[ant1]) * g[ant2] * sum_taps conj?(tap) * grid[pol][cell]
 * (conjugated taps for stacks), and 0 for dropped groups. vis_out is overwritten.
 * If grad_gains[i] is non-NULL it receives (overwritten, complex64 [nant]) the gradient of a
 * real loss with respect to the gains of the forward model w * g1 * conj(g2) * V, given that
 * grid[i] holds the gradient with respect to the grid (torch convention dL/dRe + i dL/dIm):
 *   grad_g[a] = sum_{ant1 = a} g2 conj(V) y + sum_{ant2 = a} g1 V conj(y),
 * with y the adjoint output without gains and V = vis_in[i] (required then). vis_out and
 * vis_in are 16-byte aligned with 2 or 4 polarisations (8-byte with one), like vis in mw_grid.
 * Errors: MW_ERR_INVALID_ARG (null or misaligned arrays), MW_ERR_STATE (gains for an
 * instance without antennas), MW_ERR_HIP.
 */
mw_status mw_degrid(mw_plan plan, const void *const *grid, const void *const *gains,
                    const void *const *vis_in, void *const *vis_out, void *const *grad_gains,
                    void *stream);

/*
 * Image (Section 2: images formed via a Fourier transform, one per polarisation; Section 2.1;
 * Table 1 "FFT" and "Convolution Correction"), per instance and polarisation. direction = +1:
 *   out[p] = sum_g in[g] exp(+2 pi i (g - n/2)(p - n/2)/n) in x and y (unnormalised,
 *   centred), then, if correct, out /= Cn(x) Cn(y) with Cn(x) = psi_0(c, 2x)/psi_0(c, 0),
 *   x = (p - n/2)/n (the normalised Fourier transform of the built-in kernel).
 * direction = -1 is the exact adjoint: the correction first, then the sign -i transform.
 * in and out are device complex64 [npol][ny][nx]; in == out is allowed (in place); in is
 * left unchanged otherwise. correct = 1 is rejected for instances planned with stacks.
 * Errors: MW_ERR_INVALID_ARG, MW_ERR_STATE, MW_ERR_HIP.
 */
mw_status mw_image(mw_plan plan, const void *const *in, void *const *out, int32_t direction,
                   int32_t correct, void *stream);

/*
 * Stokes conversion, per instance (Section 2.1: the instrumental-polarisation images are
 * converted to Stokes parameters by a 4 x 4 matrix that depends on time and on the pixel's
 * position relative to the instrument, at every pixel; Table 1 "Stokes Conversion").
 * images[i]: device complex64 [4][ny][nx], the XX, XY, YX, YY images as mw_image returns
 * them from visibilities gridded without their Hermitian mirror; the pixel's measured
 * coherency is then E = [[2 Re XX, XY + conj(YX)], [YX + conj(XY), 2 Re YY]].
 * jones: NULL, or jones[i] NULL (ideal feeds, J = 1) or device complex64 [ny][nx][2][2], the
 * instrument's response J toward each pixel for the snapshot's time, row-major
 * (J00, J01, J10, J11), with measured = J C J^H. The sky coherency C = J^-1 E J^-H gives
 * out[i]: device float32 [4][ny][nx] = I = (C00 + C11)/2, Q = (C00 - C11)/2, U = Re C01,
 * V = Im C01 (overwritten). A singular J gives non-finite values at its pixel (no error).
 * images and jones must be 16-byte aligned, out 8-byte aligned. FP32 arithmetic.
 * Errors: MW_ERR_INVALID_ARG (null arrays, misalignment), MW_ERR_STATE (an instance without
 * 4 polarisations), MW_ERR_HIP.
 */
mw_status mw_stokes(mw_plan plan, const void *const *images, const void *const *jones,
                    void *const *out, void *stream);

/*
 * Calibration (Section 2: the complex gain of each antenna from a linear least-squares fit to
 * observed catalogue sources; Section 2.1: the contribution of catalogue sources is measured
 * and removed in decreasing order of predicted flux, each measurement constraining the antenna
 * gains, iteratively; Table 1, "CML"). These calls use the instance's uvw and frequencies as
 * planned, every group (flags and the grid's footprint rule do not apply; pass zero weights to
 * exclude samples) and scalar gains per antenna shared by all polarisations.
 *
 * mw_predict: vis = (or +=, accumulate = 1) sum over sources of S exp(-2 pi i (u l + v m +
 * w (n - 1))), n = sqrt(1 - l^2 - m^2), (u, v, w) = uvw * f / 299792458, times
 * g[a1] conj(g[a2]) if gains is given (device complex64 [nant]; needs antennas). Unpolarised
 * sources: with 4 polarisations the cross terms XY, YX (1, 2) are zero. sources: device
 * float64 [nsrc][3] = (l, m, S). vis: device complex64 [ngroups][npol]. Phases in FP64, reduced
 * to a fraction of a turn before FP32 sine and cosine; FP32 sums.
 */
mw_status mw_predict(mw_plan plan, int32_t inst, const double *sources, int32_t nsrc,
                     const void *gains, void *vis, int32_t accumulate, void *stream);

/*
 * mw_solve_gains: per-antenna complex gains g with vis ~ g[a1] conj(g[a2]) model, by niter
 * iterations of the alternating least-squares method of Salvini & Wijnholds (2014,
 * "StEFCal"): each iteration solves every antenna's gain with the others at the previous
 * iterate, g_p = sum w z conj(R) / sum w |z|^2 over the samples involving p, and every second
 * iterate is averaged with the previous one. gains: device complex64 [nant], the starting
 * point in, the solution out (an antenna without weighted samples keeps its value). vis,
 * model: device complex64 [ngroups][npol], 16-byte aligned (8 with one polarisation); weights:
 * device float32 [ngroups] or NULL (= 1). rel_step: device float32 [1] or NULL, receives
 * ||g_i - g_(i-1)|| / ||g_i|| of the last iteration. Needs an instance planned with antennas
 * (else MW_ERR_STATE); misaligned arrays give MW_ERR_INVALID_ARG.
 */
mw_status mw_solve_gains(mw_plan plan, int32_t inst, const void *vis, const void *model,
                         const float *weights, void *gains, int32_t niter, float *rel_step,
                         void *stream);

/*
 * mw_peel: the measurement loop. Sources (host float64 [nsrc][3] = (l, m, S), read before the
 * call returns) are taken in decreasing |S|, ties in catalogue order. For each: the gains
 * toward it are solved (mw_solve_gains from unit gains, niter >= 1 iterations) from the current
 * residual against its prediction, and g[a1] conj(g[a2]) times the prediction is removed from
 * the residual. resid: device complex64 [ngroups][npol] (may equal vis; starts as vis), like
 * vis 16-byte aligned (8 with one polarisation); gains: device complex64 [nsrc][nant], row k for
 * catalogue entry k; rel_step: device float32 [nsrc] or NULL. The plan keeps a device and a
 * pinned host copy of the catalogue (grown on demand). Needs an instance planned with antennas.
 */
mw_status mw_peel(mw_plan plan, int32_t inst, const void *vis, const double *sources, int32_t nsrc,
                  const float *weights, int32_t niter, void *resid, void *gains, float *rel_step,
                  void *stream);

/*
 * w-stacking: the images of a plan's instances, one w-plane each (every instance with a
 * w-range, the same grid size, cell size and polarisations), summed with the w-term of their
 * plane: out[p] (+)= sum_k images[k][p] exp(+2 pi i w_k (n - 1)) at every pixel, with
 * w_k = (wlo + whi) / 2 of instance k, l = (x - nx/2) / (nx du), m = (y - ny/2) / (ny dv),
 * n = sqrt(1 - l^2 - m^2) (0 outside the unit circle). The images come from mw_image of each
 * plane's grid (with the convolution correction if wanted). images[k]: device complex64
 * [npol][ny][nx]; out: device complex64 [npol][ny][nx] (accumulate = 0 overwrites). At most 64
 * planes per call. Phases in FP64, reduced to a fraction of a turn before FP32 sine and
 * cosine. Errors: MW_ERR_INVALID_ARG, MW_ERR_STATE (an instance without a w-range, or
 * instances of different shapes), MW_ERR_UNSUPPORTED (more than 64 planes), MW_ERR_HIP.
 */
mw_status mw_wstack_combine(mw_plan plan, const void *const *images, void *out, int32_t accumulate,
                            void *stream);

/* Statistics and chosen launch of instance inst (inst = -1: sums over instances). */
mw_status mw_plan_info(mw_plan plan, int32_t inst, mw_plan_stats *out);

/*
 * Copy instance inst's gridding order to host memory (the sort by uv tile that stands for the
 * memory structures Section 3.2 says the port needed): order_host uint32 [nkept] = the input
 * index of each kept group in the order the gridder and degridder take them (tile, then cell,
 * then row sub-position; equal keys in input order). Synchronous. MW_ERR_INVALID_ARG: inst
 * out of range or NULL.
 */
mw_status mw_plan_order(mw_plan plan, int32_t inst, uint32_t *order_host);

/*
 * Copy instance inst's integer plan outputs to host memory: pos_host int32 [ngroups][4] =
 * cx, cy, px, py for kept groups and -1, -1, -1, -1 for dropped ones. Synchronous.
 */
mw_status mw_plan_positions(mw_plan plan, int32_t inst, int32_t *pos_host);

/*
 * Copy instance inst's kernel tables to host memory (built-in kernel only; any pointer may
 * be NULL): table_host float [O][W] (row = phase + O/2), corr_x float [nx], corr_y [ny].
 */
mw_status mw_plan_tables(mw_plan plan, int32_t inst, float *table_host, float *corr_x,
                         float *corr_y);

/*
 * Profiling of the library's own launches. With enable = 1, every later mw_grid call on the
 * plan records HIP events on its stream around the gridder kernel and the merge pass of each
 * instance (a few microseconds of overhead); enable = 0 stops it.
 */
mw_status mw_plan_set_timing(mw_plan plan, int32_t enable);

/*
 * Durations of the last timed mw_grid call of instance inst (waits for that call to
 * finish): grid_ms = the gridder kernel, merge_ms = the merge pass (0 when the launch has
 * none). Either pointer may be NULL. MW_ERR_STATE if no timed call was made.
 */
mw_status mw_plan_kernel_ms(mw_plan plan, int32_t inst, float *grid_ms, float *merge_ms);

/* Release everything the plan owns (waits for its outstanding work). NULL is a no-op. */
mw_status mw_plan_destroy(mw_plan plan);

/* Description of the last failure on the calling thread; valid until its next call. */
const char *mw_last_error(void);

/* MW_ABI_VERSION of the library. */
int32_t mw_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MWAGRID_H */
