/*
 * ivx_dataproc — the data processor that prepares the forward operator's inputs, and the
 * image-domain combination steps of the paper's pipeline, on the GPU.
 *
 *   Sect. 3.3  primary beams resampled to the pixel scale of the sky image, and for each
 *              pointing an interpolation grid giving, for every pixel of its SIN (orthographic)
 *              sub-image, the sampling location in the sky-image frame (Eq. sin_projection);
 *   Sect. 4.4.1 the inverse mapping (Eq. sin_deprojection), and linear mosaicking of
 *              per-pointing images weighted by the squared beams (Eq. linear) with the
 *              effective beam sqrt(sum_k A_k^2) (Eq. pb_eff);
 *   App. B     feathering: the single-dish map supplies the large scales through a Gaussian
 *              transfer function B(k) in Fourier space, the interferometric image the rest.
 *
 * SIN frames: an image of n x n pixels of size delta (radians) tangent at (ra, dec) has its
 * reference pixel at (row, col) = (n/2, n/2) and pixel (row, col) at direction cosines
 * l = (col - n/2) delta, m = (row - n/2) delta (l along columns, m along rows, no sign flip).
 * Coordinates are computed in FP64 and stored as ivx_real.  Status codes and
 * ivx_last_error() are those of ivx.h.  All calls are asynchronous on `stream` and allocate
 * no device memory; pointers marked device must be device memory of the current device.
 */
#ifndef IVX_DATAPROC_H
#define IVX_DATAPROC_H

#include <stdint.h>

#include "ivx.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t n;       /* image edge in pixels (>= 4) */
    int32_t reserved; /* 0 */
    double delta;    /* pixel size, radians (> 0) */
    double ra, dec;  /* tangent point, radians */
} ivx_sin_frame;

/* Interpolation grids of P pointings (Sect. 3.3, Eq. sin_projection): sub-pixel (a, b) of
 * pointing k's n_sub x n_sub SIN sub-image (pixel size sub_delta, tangent at centres[k] =
 * (ra_k, dec_k), host [P][2] radians) looks at the sky-frame position
 *   grids[k][a][b] = (row, col), device [P][n_sub][n_sub][2],
 * the input `interp` of ivx_plan_set_data. */
ivx_status ivx_dp_sin_grids(const ivx_sin_frame *sky, int32_t n_point, const double *centres, int32_t n_sub,
                            double sub_delta, ivx_real *grids, void *stream);

/* The inverse (Eq. sin_deprojection): sky pixel (i, j) is at (row, col) = grids[k][i][j] of
 * pointing k's sub-image, device [P][N][N][2] with N = sky->n.  Directions on the far side of
 * pointing k (n <= 0) get (-1e9, -1e9), outside any image. */
ivx_status ivx_dp_deprojection_grids(const ivx_sin_frame *sky, int32_t n_point, const double *centres,
                                     int32_t n_sub, double sub_delta, ivx_real *grids, void *stream);

/* Primary beams resampled to the sub-image pixel scale (Sect. 3.3): beams_in [P][nb][nb]
 * (pixel size beam_delta, reference pixel (nb/2, nb/2) at the pointing centre) ->
 * beams_out [P][n_sub][n_sub] (pixel size sub_delta): sub-pixel (a, b) at (l, m) reads the
 * input at (m / beam_delta + nb/2, l / beam_delta + nb/2), bilinear, 0 outside.  Device. */
ivx_status ivx_dp_resample_beams(int32_t n_point, const ivx_real *beams_in, int32_t nb, double beam_delta,
                                 int32_t n_sub, double sub_delta, ivx_real *beams_out, void *stream);

/* Linear mosaic (Sect. 4.4.1, Eq. linear and Eq. pb_eff) of C channels of P per-pointing
 * images: for every sky pixel r, with I'_kc(r) and A_k(r) the bilinear samples of
 * sub_images[k][c] ([P][C][n_sub][n_sub]) and beams[k] ([P][n_sub][n_sub]) at
 * deproj[k][r] (from ivx_dp_deprojection_grids, [P][N][N][2]),
 *   image[c][r] = sum_k A_k(r)^2 I'_kc(r) / sum_k A_k(r)^2   where A_eff(r) >= pb_min, else 0,
 *   pb_eff[r]   = A_eff(r) = sqrt(sum_k A_k(r)^2)            (pb_eff may be NULL).
 * image [C][N][N].  Device memory. */
ivx_status ivx_linear_mosaic(int32_t n_point, int32_t n_chan, int32_t n_sub, const ivx_real *sub_images,
                             const ivx_real *beams, int32_t n_sky, const ivx_real *deproj, double pb_min,
                             ivx_real *image, ivx_real *pb_eff, void *stream);

/* Bytes of the `work` buffer ivx_feather needs for C channels of n x n maps. */
int64_t ivx_feather_work_bytes(int32_t n_chan, int32_t n);

/* Feathering (App. B): for each channel,
 *   out = F^-1[ B(k) F[single_dish] + (1 - B(k)) F[interf] ],
 *   B(k) = exp(-2 pi^2 sigma^2 |k|^2), sigma = theta / (2 sqrt(2 ln 2)),
 * with k the spatial frequency of the n x n grid of pixel size delta (cycles per radian:
 * (p, q) / (n delta), p and q the signed FFT frequency indices).  Both maps are on the same
 * pixel grid and in the same units (a brightness-temperature map is converted with the
 * Rayleigh-Jeans relation by the caller).  interf, single_dish, out: device [C][n][n];
 * out may alias interf.  n: power of two in [64, 2048].  work: device, at least
 * ivx_feather_work_bytes(C, n) bytes, contents undefined afterwards. */
ivx_status ivx_feather(int32_t n_chan, int32_t n, double delta, double theta, const ivx_real *interf,
                       const ivx_real *single_dish, ivx_real *out, void *work, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* IVX_DATAPROC_H */
