/*
 * ivx — objective and gradient of the Classic3D joint-deconvolution criterion on one
 * MI355X (gfx950).  C ABI: plain pointers and sizes, no C++ or framework types.
 *
 * What is evaluated (Sect. 2.1, 2.2, 2.4; Eq. Q, Eq. 3, Eq. fusion_cost):
 *
 *   Q_tot(x) = sum_{k,c} J_kc(x) + lambda_s sum_c K_c(x) + lambda_r sum_c R_c(x)
 *              + lambda_nu R_nu(x)
 *
 *   J_kc = 1/2 sum_j w_j | V_j - y_j |^2   over the unflagged visibilities of pointing k,
 *          channel c, with w_j = 1/sigma_j^2 (the SIGMA column, Sect. 2.2) and the model
 *   V_j  = sum_{a,b} s_c A_k[a][b] x'_kc[a][b] exp(-2 pi i (u_j l_b + v_j m_a))
 *          (coplanar forward model, Sect. 2.1), l_b = (b - n/2) delta along columns,
 *          m_a = (a - n/2) delta along rows, n = n_sub;
 *   x'_kc = bilinear sample of sky channel c on pointing k's interpolation grid
 *          (SIN reprojection, Eq. sin_projection; grids precomputed, Sect. 3.3):
 *          sub-pixel (a,b) reads sky coordinate (row, col) = interp[k][a][b][0..1],
 *          sky pixel (i,j) sits at coordinate (i,j), pixels outside [0,N)^2 read 0;
 *   R_c  = 1/2 || D x_c ||^2, D = 3x3 Laplacian [[0,-1,0],[-1,4,-1],[0,-1,0]] with zero
 *          padding (Eq. 3);
 *   K_c  = 1/2 sum_{p,q} ((T~_c[p][q] - T_c[p][q]) / sigma_sd)^2, T~ = the sky convolved
 *          with a unit-sum Gaussian single-dish beam (FWHM sd_fwhm_rad, truncated at
 *          4 sigma, zero padding), point-sampled at rows/cols sd_offset + p*sd_stride
 *          (fusion term, Sect. 2.4).
 *   R_nu = 1/2 sum_{c=0}^{C-2} || x_{c+1} - x_c ||^2, a spectral smoothness term coupling
 *          adjacent channels (an extension of the regulariser family of Sect. 2.2-2.3; the
 *          paper's own solves keep channels independent, lambda_nu = 0).
 *
 * The gradient returned is dQ_tot/dx over the whole cube, in the same layout as x.
 * The visibility model is evaluated with a non-uniform FFT (exponential-of-semicircle
 * kernel, Barnett et al. 2019 — the paper's NUFFT reference, Sect. 2.1) whose accuracy is
 * set by nufft_eps or an explicit kernel width; all work runs in hand-written gfx950
 * kernels.  The floating-point type of every real array below is ivx_real: float in
 * libivx.so, double in the FP64 test build libivx_f64.so (same symbols).
 *
 * Layouts (all row-major, C order):
 *   sky, grad, image    [n_chan][n_sky][n_sky]
 *   uv                  [M][2]  (u, v) in wavelengths, ivx_real
 *   vis, model_vis      [M][2]  (re, im) interleaved, ivx_real
 *   weight              [M]     ivx_real, natural weights 1/sigma^2
 *   flags               [M]     uint8, non-zero = flagged (dropped at set_data), or NULL
 *   beams               [n_point][n_sub][n_sub]       ivx_real, primary beam A_k
 *   interp              [n_point][n_sub][n_sub][2]    ivx_real, (row, col) sky coordinate
 *   sd_map              [n_chan][sd_n][sd_n]          ivx_real, or NULL
 *   The M visibilities are stored block after block, block b = k * n_chan + c
 *   (pointing-major); vis_offsets[b] .. vis_offsets[b+1] is block b.
 *
 * Memory: every pointer argument may be host memory or device memory of the current
 * device (the library copies with hipMemcpyDefault).  The caller keeps ownership of
 * everything it passes; set_data copies, compacts and reorders what it needs into plan-
 * owned device memory, so caller buffers may be freed as soon as it returns.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = the default stream).  All
 * evaluation calls are asynchronous on that stream except where a host pointer receives
 * results (terms), which synchronises the stream.
 *
 * Errors: every call returns an ivx_status; a negative value means nothing was written
 * to the caller's outputs.  ivx_last_error() gives a thread-local message for the last
 * failure.  No C++ exception crosses this boundary.  Calls on one plan are not
 * re-entrant: one plan must not be used from two threads at once.
 */
#ifndef IVX_H
#define IVX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#ifdef IVX_REAL_DOUBLE
typedef double ivx_real;
#else
typedef float ivx_real;
#endif

#define IVX_VERSION 5

typedef enum {
    IVX_OK = 0,
    IVX_EINVAL = -1,     /* bad shape, size, pointer or parameter */
    IVX_ENOMEM = -2,     /* device or host allocation failed; plan left unallocated */
    IVX_EHIP = -3,       /* HIP runtime error (message in ivx_last_error) */
    IVX_ENONFINITE = -4, /* NaN/Inf found in unflagged input data by set_data */
    IVX_ESTATE = -5      /* call out of order (e.g. evaluation before set_data) */
} ivx_status;

typedef struct ivx_plan ivx_plan;

/* Problem geometry and hyper-parameters (Sect. 2.2 lambda_r, Sect. 2.4 lambda_s). */
typedef struct {
    int32_t n_chan;             /* C >= 1 spectral channels */
    int32_t n_sky;              /* N: sky is N x N pixels */
    double pixel_rad;           /* delta > 0: pixel size of sky and sub-images, radians */
    int32_t n_point;            /* P >= 1 pointings */
    int32_t n_sub;              /* n: sub-image size (even, >= 4); phase centre (n/2, n/2) */
    const int64_t *vis_offsets; /* host, P*C+1 non-decreasing entries, [0] = 0 */
    const double *flux_scale;   /* host, [C]: s_c, sky units -> Jy per pixel */
    double lambda_r;            /* Laplacian regularisation weight, >= 0 */
    double lambda_s;            /* single-dish fusion weight, >= 0 (0 ignores sd_map) */
    int32_t sd_n;               /* single-dish map is sd_n x sd_n (0 = no fusion term) */
    int32_t sd_stride;          /* sampling stride in sky pixels */
    int32_t sd_offset;          /* first sample row/column */
    double sd_fwhm_rad;         /* single-dish beam FWHM, radians */
    double sd_sigma;            /* single-dish noise sigma_sd > 0 */
    double nufft_eps;           /* requested NUFFT accuracy (0 = 1e-7 float, 1e-12 double) */
    int32_t kernel_width;       /* spreading kernel width in fine cells (0 = from eps) */
    int32_t fine_size;          /* fine grid n_f, power of two >= 2 n_sub (0 = auto) */
    int32_t tile;               /* gridding tile edge in fine cells (0 = auto) */
    int32_t reserved;           /* must be 0 */
    double lambda_nu;           /* spectral smoothness weight, >= 0 (0 = channels independent) */
} ivx_problem;

/* Validate `d`, choose the NUFFT parameters and allocate the plan.  No device memory is
 * touched until set_data.  *out is NULL on failure. */
ivx_status ivx_plan_create(const ivx_problem *d, ivx_plan **out);

/* Copy the data of every block into the plan (Sect. 3.2: all pointings concatenated):
 * drops flagged visibilities, folds u<0 onto u>0 by Hermitian symmetry of a real sky,
 * sorts by fine-grid tile and builds the work list, on the device, one block at a time
 * (host arrays are staged block by block, so host inputs need no device copy of the whole
 * data set).  beams and interp are required; flags and sd_map may be NULL (sd_map is
 * required when lambda_s > 0 and sd_n > 0).  Every block must hold fewer than 2^31
 * visibilities (IVX_EINVAL otherwise).  Returns IVX_ENONFINITE if an unflagged
 * visibility, weight or uv is not finite, IVX_EINVAL if a weight is negative (whichever
 * comes first in caller order).  May be called again to replace the data (same sizes).
 * Device memory kept: 20 B (float build; 28 B FP64) per live visibility plus the grids. */
ivx_status ivx_plan_set_data(ivx_plan *plan, const ivx_real *uv, const ivx_real *vis,
                             const ivx_real *weight, const uint8_t *flags,
                             const ivx_real *beams, const ivx_real *interp,
                             const ivx_real *sd_map, void *stream);

/* As ivx_plan_set_data for a spectral cube whose channels share one uv track per
 * pointing (Sect. 2.1, Eq. vis: each channel's model uses the pointing's baselines in
 * wavelengths at that channel's frequency, so one track scaled by nu_c / nu_ref serves
 * every channel):
 *   uv      [sum_k M_k][2]  pointing k's samples at rows pt_k .. pt_k + M_k - 1 (pointing
 *                           order), in wavelengths at a reference frequency
 *   weight  [sum_k M_k]     natural weights, the same for every channel
 *   uv_scale[C]             host; channel c sees uv * uv_scale[c] (nu_c / nu_ref), > 0
 *   vis     [M][2], flags [M] (or NULL): per (pointing, channel) block as in set_data
 * Every channel of pointing k must have M_k visibilities in vis_offsets (IVX_EINVAL
 * otherwise).  ivx_plan_set_vis on such a plan takes weights in the [sum_k M_k] layout. */
ivx_status ivx_plan_set_data_shared(ivx_plan *plan, const ivx_real *uv, const ivx_real *weight,
                                    const double *uv_scale, const ivx_real *vis,
                                    const uint8_t *flags, const ivx_real *beams,
                                    const ivx_real *interp, const ivx_real *sd_map, void *stream);

/* The full forward model of Sect. 2.1, Eq. vis: every pixel of a sub-image also carries the
 * factor 1/n and the phase w (n - 1), n = sqrt(1 - l^2 - m^2) of pixel (a, b):
 *   V_j = sum_{a,b} s_c A_k x'_kc[a][b] / n_ab exp(-2 pi i (u_j l_b + v_j m_a + w_j (n_ab - 1))).
 * The coplanar model above is its small-angle form, whose phase error grows as pi |w| theta^2
 * with the distance theta from the phase centre (Sect. 2.1).
 *   w        [M] (or [sum_k M_k] for a plan set with ivx_plan_set_data_shared, scaled by
 *            uv_scale[c] like uv), wavelengths, caller order, host or device; NULL returns the
 *            plan to the coplanar model.
 *   w_width  w kernel width in planes, 0: max(the plan's kernel width, 8); 2..16.
 *   w_sigma  oversampling of the w planes, 0: 2.0; 1.25..8.
 * After this call ivx_objective_grad, ivx_objective, ivx_objective_forward / _backward,
 * ivx_forward, ivx_adjoint and ivx_forward_adjoint evaluate the full model: w-stacking over
 * planes w_p = w0 + p dw, dw = 1 / (w_sigma X) (X the range of n - 1 over the sub-image),
 * interpolated in w with the same exponential-of-semicircle kernel and deapodized by its
 * Fourier transform, so the w direction reaches the (u, v) transform's accuracy at that
 * oversampling.  Cost per evaluation: one complex FFT pair per plane and block (the widest
 * block's plane count, ivx_plan_w_info) plus w_width passes over every visibility each way;
 * evaluations run as eager launches (no captured graph).  Device memory added: 12 B (float
 * build; 24 B FP64) per live visibility, one n_sub x extended-column complex buffer per block,
 * a copy of w, and three n_sub^2 tables.
 * Errors: IVX_ESTATE before a successful set_data (set_data drops the w coordinates: call
 * again after it); IVX_EINVAL for a width or oversampling out of range, a sub-image pixel
 * outside the unit circle, a block spanning more than 255 planes, or work items longer than
 * 2048 visibilities (choose a smaller chunk with ivx_set_blocking); IVX_ENONFINITE if an
 * unflagged w is not finite.  On failure the plan keeps the coplanar model. */
ivx_status ivx_plan_set_w(ivx_plan *plan, const ivx_real *w, int32_t w_width, double w_sigma, void *stream);

/* Geometry of the full model: info[6] = {enabled (0/1), planes of the widest block, dw
 * (wavelengths), x_c (the centre of the n - 1 range), w_width, w_sigma}. */
ivx_status ivx_plan_w_info(const ivx_plan *plan, double *info);

/* Replace the visibility data (and, if `weight` is non-NULL, the weights) of a plan whose
 * uv coverage, flags, beams and grids stay the same: vis [M][2] and weight [M] (or
 * [sum_k M_k] for a shared-uv plan) in the caller's order, host or device memory.  The
 * reordering runs on the device; IVX_ENONFINITE if an unflagged value is not finite or a
 * weight is negative (checked on the device, then the stream is synchronised).  Same
 * observation, new data: no re-sort. */
ivx_status ivx_plan_set_vis(ivx_plan *plan, const ivx_real *vis, const ivx_real *weight,
                            void *stream);

/* One evaluation of Q_tot and its gradient at sky x (Eq. fusion_cost).
 * sky, grad: device, [C][N][N]; grad is overwritten.  terms (host or device, 4 doubles)
 * receives {Q_tot, Q, K, R} with Q = sum J_kc; NULL skips it.  Host `terms`
 * synchronises the stream. */
ivx_status ivx_objective_grad(ivx_plan *plan, const ivx_real *sky, ivx_real *grad,
                              double *terms, void *stream);

/* The objective and its gradient as two halves, for a reverse-mode caller (the paper obtains
 * the gradient of Q_tot by automatic differentiation, Sect. 3.4; here the reverse pass is the
 * hand-written adjoint):
 *   ivx_objective           Q_tot terms only (no gradient work: nothing is spread).
 *   ivx_objective_forward   the terms, and the weighted residuals spread into the plan's
 *                           per-tile windows (the forward model, residual and data term share
 *                           one pass over the visibilities with the spread).
 *   ivx_objective_backward  the rest of the gradient from those windows: inverse FFTs, beam
 *                           and reprojection transpose summed over pointings, regulariser and
 *                           single-dish gradients, all multiplied by `scale` (the incoming
 *                           gradient of the caller's loss with respect to Q_tot).
 * forward + backward(scale = 1) gives the terms and gradient of ivx_objective_grad (the same
 * sums).  backward needs the same `sky` pointer as the forward it follows and no other call on
 * the plan in between (IVX_ESTATE otherwise); it consumes the windows, so each forward allows
 * one backward.  terms: 4 doubles {Q_tot, Q, K, R}, host (synchronises) or device. */
ivx_status ivx_objective(ivx_plan *plan, const ivx_real *sky, double *terms, void *stream);
ivx_status ivx_objective_forward(ivx_plan *plan, const ivx_real *sky, double *terms, void *stream);
ivx_status ivx_objective_backward(ivx_plan *plan, const ivx_real *sky, ivx_real *grad, double scale,
                                  void *stream);

/* Model visibilities V(sky) of every block in the caller's original order (flagged
 * entries are written as 0).  sky: device [C][N][N]; model_vis: device [M][2]. */
ivx_status ivx_forward(ivx_plan *plan, const ivx_real *sky, ivx_real *model_vis,
                       void *stream);

/* Weighted adjoint: image = Re sum_k P_k^T s_c A_k F^H W v  (flagged entries ignored),
 * the transpose of ivx_forward with the natural weights; it equals -grad Q at x = 0
 * when v = y.  vis: device [M][2] caller order; image: device [C][N][N], overwritten. */
ivx_status ivx_adjoint(ivx_plan *plan, const ivx_real *vis, ivx_real *image, void *stream);

/* Transpose of ivx_forward without weights (the vector-Jacobian product of the forward model,
 * Sect. 2.1): image = Re sum_k P_k^T s_c A_k F^H v for v in the caller's order ([M][2]; flagged
 * entries ignored).  For a cotangent g of the model visibilities, <g, ivx_forward(x)> =
 * <image, x>.  vis: device [M][2]; image: device [C][N][N], overwritten. */
ivx_status ivx_forward_adjoint(ivx_plan *plan, const ivx_real *vis, ivx_real *image, void *stream);

/* Time whole evaluations of this plan's data (at a zero sky) for candidate blockings (tile
 * edge, waves per block, visibilities per work item, gridder variant) that fit the LDS, and
 * keep the fastest.  When the plan was created with kernel_width = 0 and fine_size = 0, the
 * candidates also cover NUFFT geometries: on the plan's fine grid and on grids of half and
 * twice its size, the narrowest kernel whose accuracy probe (ivx_nufft_probe) meets the
 * plan's target -- nufft_eps when it was given, else the probe value of the plan's own
 * geometry -- so the choice never makes the transform less accurate than that target.
 * Blockings alone are accuracy-neutral.  budget_ms bounds the time spent; *chosen_tile
 * (host, may be NULL) receives the tile edge kept; ivx_plan_info reports the kernel width
 * and fine grid. */
ivx_status ivx_autotune(ivx_plan *plan, double budget_ms, int32_t *chosen_tile, void *stream);

/* Accuracy probe of a NUFFT geometry (sub-image edge n_sub, fine grid n_fine, kernel width):
 * the largest error, over the sub-image frequencies and positions within one fine cell, of
 * the one-dimensional transform of a unit point source computed with the library's spreading
 * kernel and deapodization, against its closed form exp(-2 pi i k x / n_fine) (Sect. 2.1's
 * model for one source).  The two-dimensional error is at most about twice this. */
ivx_status ivx_nufft_probe(int32_t n_sub, int32_t n_fine, int32_t kernel_width, double *err);

/* Stable radix sort of unsigned 64-bit keys on their bits [0, end_bit) (end_bit 1..64),
 * optionally carrying one 32-bit value per key: the device sort behind the plan's binning
 * of the visibility records (Sect. 2.3's gridding by tile) and behind the bounded solver's
 * ordering of the breakpoints of the generalized Cauchy point (Sect. 3.4, Eq. L-BFGS-B).
 * keys_in / keys_out (and vals_in / vals_out) are caller-owned device arrays of n entries
 * that must not overlap; vals_in = NULL sorts keys only and ignores vals_out.  Keys that
 * agree on the sorted bits keep their input order.  The call allocates and frees its own
 * scratch (the plan and the solver keep theirs) and synchronises `stream`.  IVX_EINVAL for
 * n outside [0, 2^31), end_bit outside 1..64 or a missing array; n = 0 does nothing. */
ivx_status ivx_sort_u64(const uint64_t *keys_in, uint64_t *keys_out, const uint32_t *vals_in,
                        uint32_t *vals_out, int64_t n, int32_t end_bit, void *stream);

/* ivx_objective_grad records its launches into a HIP graph on first use and replays it
 * while the (sky, grad) pointers stay the same (a new pair re-captures).  enable = 0
 * launches the kernels one by one instead; results are identical. */
ivx_status ivx_set_graph(ivx_plan *plan, int enable);

/* Stages of one evaluation, in launch order (bit i of a stage mask = stage i). */
enum {
    IVX_STAGE_IMAGE_ROWS = 0, /* reprojection x beam x deapodization + row FFTs */
    IVX_STAGE_COL_FWD = 1,    /* column FFTs -> extended fine grid */
    IVX_STAGE_GRID = 2,       /* degrid, residual, data term, spread (per tile) */
    IVX_STAGE_FOLD = 3,       /* slot reduction + Hermitian symmetrisation */
    IVX_STAGE_COL_INV = 4,    /* inverse column FFTs */
    IVX_STAGE_ROW_INV = 5,    /* inverse row FFTs x deapodization x beam */
    IVX_STAGE_SD = 6,         /* single-dish model and residual */
    IVX_STAGE_SKY = 7,        /* reprojection transpose + Laplacian + single-dish gradient */
    IVX_STAGE_FINAL = 8,      /* FP64 reduction of the four terms */
    IVX_NSTAGE = 9
};

/* Device timing of ivx_objective_grad: while stage_mask != 0, each evaluation records a
 * HIP event pair on the evaluation stream around every stage in the mask.  The events
 * are owned by the plan.  ivx_stage_times waits for them, writes the summed milliseconds
 * per stage into ms[IVX_NSTAGE] (host) and the number of timed evaluations into *n_eval
 * (host), and resets the sums. */
ivx_status ivx_set_timing(ivx_plan *plan, uint32_t stage_mask);
ivx_status ivx_stage_times(ivx_plan *plan, double *ms, int64_t *n_eval);

/* Set the gridding blocking explicitly instead of ivx_autotune: tile edge (>= kernel
 * width), waves per block (1, 2 or 4), visibilities per work item (>= 16), lanes per
 * visibility (16, or 8 when kernel_width <= 8) and visibilities per lane group per loop
 * iteration (1 or 2).  IVX_EINVAL if the combination does not fit the LDS; results are
 * identical for every accepted blocking. */
ivx_status ivx_set_blocking(ivx_plan *plan, int32_t tile, int32_t waves, int32_t chunk,
                            int32_t lanes, int32_t vpi, void *stream);

/* Register budget of the matrix-core gridder (blockings with 64 lanes per visibility): the
 * build compiled for 6 or 7 resident waves per SIMD, or 0 (the default) to use 7 from
 * 32,768 work items up and 6 below.  Results are identical for both builds (same
 * arithmetic in the same order); only the schedule changes.  IVX_EINVAL otherwise. */
ivx_status ivx_set_gridder_occupancy(ivx_plan *plan, int32_t waves_per_simd);

/* Adjoint of the gridding stage: the per-tile windows are either summed straight into the
 * inverse column FFT (one kernel; IVX_STAGE_FOLD then takes no time) or written to the
 * extended grid by the fold and read back by the column pass.  enable = 1 (the default) fuses
 * where the fine grid allows it and the plan has enough (pointing, channel) blocks for the
 * fused launch to be faster (mosaics, cubes); 2 fuses wherever the grid allows; 0 never.
 * Results are identical (the same sums in the same order).  IVX_EINVAL otherwise. */
ivx_status ivx_set_fused_fold(ivx_plan *plan, int enable);

/* Plan facts, host array of 16 int64: {n_fine, kernel_width, tile, n_work_items,
 * n_live_vis, n_slots, device_bytes, n_items, ext_rows, ext_cols, graph_nodes,
 * window, waves_per_block, max_vis_per_work_item, lanes_per_visibility,
 * visibilities_per_group_iteration}. */
ivx_status ivx_plan_info(const ivx_plan *plan, int64_t *info16);

/* The terms of the last evaluation on the plan's stream, host array of 5 doubles: {Q_tot, Q,
 * K, R, R_nu} (the evaluation calls return the first four).  Synchronises `stream`. */
ivx_status ivx_last_terms(ivx_plan *plan, double *terms5, void *stream);

/* Release every resource of the plan (NULL is accepted). */
ivx_status ivx_plan_destroy(ivx_plan *plan);

/* Thread-local description of the last failure ("" if none). */
const char *ivx_last_error(void);

/* IVX_VERSION of the library; sizeof(ivx_real) is returned by ivx_real_size(). */
int ivx_version(void);
int ivx_real_size(void);

#ifdef __cplusplus
}
#endif

#endif /* IVX_H */
