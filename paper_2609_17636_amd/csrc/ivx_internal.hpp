// Internal types shared by the plan code (ivx_api.hip) and the kernels (ivx_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ivx.h"

namespace ivx {

typedef ivx_real real;

struct alignas(2 * sizeof(real)) cpx {
    real re, im;
};

// Sorted-visibility coordinates.  Each visibility stores the fine-grid cell where its
// w x w kernel footprint starts, relative to its tile origin, and the fractional offset
// of the footprint (so every tap distance is exact to the precision of real).
//   float build : 8.24 fixed point per axis, (cell << 24) | round(frac * 2^24)
//   double build: separate integer cell and FP64 fraction
#ifdef IVX_REAL_DOUBLE
struct VisCoord {
    uint32_t ix, iy;
    double fx, fy;
};
#else
struct VisCoord {
    uint32_t xq, yq;
};
#endif

// One unit of gridding work: up to `count` visibilities of one fine-grid tile of one
// (pointing, channel) block, accumulated into its own window-sized slot.
struct WorkItem {
    int32_t item;   // block index b = k * n_chan + c
    int32_t ty, tx; // tile coordinates in the extended grid
    int32_t count;  // number of visibilities
    int64_t begin;  // first sorted visibility
    int32_t slot;   // accumulator slot index
    int32_t pad;
};

// Entry of the sky-pixel -> sub-pixel transpose of the bilinear reprojection.
struct CsrEnt {
    int32_t off; // k * n_chan * n_sub^2 + a * n_sub + b (add c * n_sub^2 for channel c)
    real w;      // bilinear weight
};

// Plan geometry passed by value to kernels.
struct Geom {
    int C, P, N;          // channels, pointings, sky edge
    int nk;               // sub-image edge (even)
    int nf, logn;         // fine grid edge (power of two) and log2
    int rw;               // nf/2 + 1 stored half-plane columns
    int W, O;             // kernel width, extended-grid offset
    real beta;            // ES kernel shape
    int T, win, ldw;      // tile edge, window edge T+W-1, LDS window row stride
    int eh, ew;           // extended grid rows / columns
    int nty, ntx;         // tiles per block along rows / columns
    int64_t r_stride;     // nk * rw   (row-FFT buffers per block)
    int64_t ext_stride;   // eh * ew   (extended grid per block)
    int64_t hs_stride;    // nf * rw   (Hermitian half-plane per block; layout reference)
    int64_t win_stride;   // win * win (slot size)
};

// Gridding modes: the objective (degrid, residual, data term, spread), the forward model
// alone, the adjoint alone (spread of given visibilities), and the data term alone (degrid
// and residual, nothing spread: an objective value without its gradient).  The two w-plane
// modes serve the w-stacked full model: degrid one w plane and add it, weighted by the
// visibility's w kernel, to a per-record accumulator (MODE_WFWD); spread per-record
// coefficients times the w kernel into one w plane (MODE_WADJ).
enum GridMode { MODE_OBJ = 0, MODE_FWD = 1, MODE_ADJ = 2, MODE_VAL = 3, MODE_WFWD = 4, MODE_WADJ = 5 };

// w coordinate of a sorted record in units of w planes, zeta = (w - w0_b) / dw, with w folded
// like the record (negated when (u, v) was): float build 8.24 fixed point (plane index in the
// top 8 bits), double build plain double.
#ifdef IVX_REAL_DOUBLE
typedef double WZ;
#else
typedef uint32_t WZ;
#endif
constexpr int WZ_MAX_PLANES = 255; // planes a block may span (float build: 8-bit plane index)

// One w plane of a w-stacked gridding pass: the records' plane coordinates (sorted within each
// work item), the per-record accumulator (MODE_WFWD) or coefficients (MODE_WADJ), the plane
// index and the w kernel (width W in planes, shape beta).
struct WPlane {
    const WZ *wz;
    cpx *acc;
    const cpx *q;
    int plane;
    int W;
    double beta;
    // optional per-work-item table of record counts below each half plane: cnt[wid * ncnt + h]
    // = records of work item wid with zeta < h / 2, h = 0 .. ncnt - 1 (NULL: binary searches)
    const int32_t *cnt;
    int ncnt;
    // adjoint pass: per slot, 1 if its work item has records near the plane (window written),
    // 0 if not (window left as it was: the fold skips it); NULL: every window is written
    uint8_t *sact;
};

// Sky pass tiling: blocks of SKY_T x SKY_T pixels, 256 threads, thread t at row t / SKY_T,
// column t % SKY_T of the block; the reprojection transpose is stored per wave ("slice":
// 64 consecutive threads) in entry-major order.
constexpr int SKY_T = 16;

// ---------------------------------------------------------------- kernel launchers
// Each returns hipSuccess or the launch error.  All run on `st`.

hipError_t launch_image_rows(const Geom &g, const real *sky, const real *beams,
                             const real *interp, const real *fscale, const real *dq,
                             const cpx *tw, cpx *R, hipStream_t st);
hipError_t launch_col_fwd(const Geom &g, const cpx *R, const cpx *tw, cpx *ext, hipStream_t st);
// perm: caller index of each sorted record within its block (bit-inverted when folded);
// boff: caller offset of every block (forward / adjoint modes only)
hipError_t launch_grid(int mode, const Geom &g, const WorkItem *work, int n_work,
                       const VisCoord *crd, const cpx *vis, const real *wgt,
                       const int32_t *perm, const int64_t *boff, const cpx *ext, cpx *slots, double *jpart,
                       const cpx *caller_in, cpx *caller_out, int nwave, int variant,
                       int occupancy, hipStream_t st, bool unweighted = false);
// adjoint extended grid: the windows summed into `ext` (the forward extended grid, which
// the gridding pass has consumed by then)
// sact (may be NULL: every slot counts) flags the slots whose windows were written; the others
// are skipped, which adds nothing to any cell (the sums are those of the written windows)
hipError_t launch_fold(const Geom &g, const int32_t *tslot, const cpx *slots, cpx *ext, hipStream_t st,
                       const uint8_t *sact = nullptr);
// inverse column FFT of the symmetrised half plane, folded from the adjoint extended grid
hipError_t launch_col_inv(const Geom &g, const cpx *E, const cpx *tw, cpx *R, hipStream_t st);
// The slot fold and the inverse column pass in one kernel (no extended grid written); only for
// grids where fold_fusable(g) holds (every cell has at most two row aliases and one column
// alias); fold_fusion_pays(g): the launch has enough (item, column group) blocks to be faster.
bool fold_fusable(const Geom &g);
bool fold_fusion_pays(const Geom &g);
hipError_t launch_col_inv_slots(const Geom &g, const int32_t *tslot, const cpx *slots, const cpx *tw, cpx *R,
                                hipStream_t st);
hipError_t launch_row_inv(const Geom &g, const cpx *R, const real *beams, const real *fscale,
                          const real *dq, const cpx *tw, real *gp, hipStream_t st);
hipError_t launch_sd_rows(const Geom &g, const real *sky, const real *gB, int rb, int sd_n,
                          int stride, int offset, real *U, hipStream_t st);
hipError_t launch_sd_cols(const Geom &g, const real *U, const real *gB, int rb, int sd_n,
                          int stride, int offset, const real *sdmap, real inv_var, real *E,
                          double *kpart, hipStream_t st);
// V[c][p][j] = sum_q g(o + q S - j) E[c][p][q] (column half of the single-dish adjoint)
hipError_t launch_sd_back(const Geom &g, const real *E, const real *gB, int rb, int sd_n, int stride, int offset,
                          real *V, hipStream_t st);
// Sky pass modes: the whole gradient and R; the reprojection transpose alone (adjoint); R
// alone (no gradient written).  The gradient is multiplied by `scale`.
enum SkyMode { SKY_FULL = 0, SKY_ADJOINT = 1, SKY_VALUE = 2 };
// lambda_nu != 0 adds the spectral term (channels c - 1 and c + 1 of the sky are read) and its
// per-block values go to npart (one double per sky block, like rpart).
hipError_t launch_sky(const Geom &g, const real *sky, const real *gp, const int32_t *cptr,
                      const CsrEnt *cent, real lambda_r, real lambda_s, const real *E,
                      const real *gB, int rb, int sd_n, int stride, int offset, real *grad,
                      double *rpart, int mode, real scale, hipStream_t st, real lambda_nu = real(0),
                      double *npart = nullptr);
int sky_blocks(const Geom &g);
// FP64 reduction of all partials into {Q_tot, Q, K, R} (terms, and terms_user if non-null).
// jpart: per-work-item partials of J; scratch: final_scratch(nj) doubles (may be 0)
int final_scratch(int nj);
// terms receives {Q_tot, Q, K, R, R_nu} (5 doubles), terms_user the first four.
hipError_t launch_final(const double *jpart, int nj, double *scratch, const double *rpart, int nr,
                        const double *kpart, int nkp, const double *npart, int nnp, double lambda_r,
                        double lambda_s, double lambda_nu, double *terms, double *terms_user, hipStream_t st);
hipError_t launch_zero(void *p, int64_t bytes, hipStream_t st);

// ---------------------------------------------------------------- plan-time binning
// Fine-grid geometry of the footprint computation (pixel size, fine grid edge, half kernel
// width, extended-grid offset) and the tiling the records are sorted for.
struct BinGeom {
    double delta, nf, hw;
    int O, T, ntx;
};
hipError_t launch_count_live(const uint8_t *flags, int64_t n, unsigned long long *out, hipStream_t st);
// keys[j] = (tile << 32) | j of sample j of a block (all ones when flagged or bad); uv is
// multiplied by `scale`; bad[0] / bad[1]: smallest gbase + j that is non-finite / has a
// negative weight (atomicMin, start from all ones)
hipError_t launch_bin_keys(int64_t n, const real *uv, double scale, const real *vis, const real *w,
                           const uint8_t *flags, const BinGeom &b, int64_t gbase, uint64_t *keys,
                           unsigned long long *bad, hipStream_t st);
// records of the first n sorted keys; counts[tile] += 1 per record
hipError_t launch_bin_emit(int64_t n, const uint64_t *keys, const real *uv, double scale, const real *vis,
                           const real *w, const BinGeom &b, VisCoord *crd, cpx *svis, real *swgt, int32_t *perm,
                           int32_t *counts, hipStream_t st);
// keys of a block's records for tile edge T_new (tstart: the block's old tile prefix)
// A change of the fine grid and kernel width as well (frac != nullptr): each record's fine-grid
// position g = footprint start - 1 - O + frac + W/2 is recovered, scaled by nf_new / nf_old and
// split again for the new width; the new fractions go to frac (x, y).
struct Regeom {
    double ratio;          // nf_new / nf_old
    double hw_old, hw_new; // W / 2
    int O_old, O_new;      // extended-grid offsets
};
hipError_t launch_rekey(int64_t n, const VisCoord *crd, const int32_t *perm, const int32_t *tstart, int ntiles_old,
                        int ntx_old, int T_old, int ntx_new, int T_new, uint64_t *keys, uint32_t *vals, int2 *foot,
                        hipStream_t st, const Regeom *rg = nullptr, double2 *frac = nullptr);
hipError_t launch_rebin_emit(int64_t n, const uint64_t *keys, const uint32_t *vals, const int2 *foot,
                             const VisCoord *crd, const cpx *vis, const real *wgt, const int32_t *perm, int ntx,
                             int T, VisCoord *crd_o, cpx *vis_o, real *wgt_o, int32_t *perm_o, int32_t *counts,
                             hipStream_t st, const double2 *frac = nullptr);
// sorted data of one block from the caller's block arrays (w may be NULL: weights kept)
hipError_t launch_gather_block(int64_t n, const int32_t *perm, const real *vis, const real *w, cpx *svis,
                               real *swgt, unsigned int *bad, hipStream_t st);
// Stable radix sort (ivx_sort.hip) of n 64-bit keys over bits [0, end_bit), with 32-bit values
// when vin != NULL; kin / kout (vin / vout) must not overlap; temp holds
// radix_sort_temp_bytes(n, vin != NULL) bytes.
size_t radix_sort_temp_bytes(int n, bool pairs);
hipError_t radix_sort(void *temp, size_t temp_bytes, const uint64_t *kin, uint64_t *kout, const uint32_t *vin,
                      uint32_t *vout, int n, int end_bit, hipStream_t st);
// radix sorts over bits [0, end_bit) for the binning; temp == NULL queries temp_bytes
hipError_t sort_keys(void *temp, size_t &temp_bytes, const uint64_t *in, uint64_t *out, int n, int end_bit,
                     hipStream_t st);
hipError_t sort_pairs(void *temp, size_t &temp_bytes, const uint64_t *kin, uint64_t *kout, const uint32_t *vin,
                      uint32_t *vout, int n, int end_bit, hipStream_t st);

// Geometry of the w-stacked full model, passed by value to its kernels.
struct WGeom {
    const int32_t *np;  // [n_items] planes of each block (0: no live visibility)
    const double *w0;   // [n_items] w of plane 0 of each block (wavelengths)
    const double *xp;   // [nk^2] x' = (n - 1) - x_c of every sub-image pixel
    const double *tp;   // [nk^2] dw x'
    const real *corr;   // [nk^2] 1 / (n Phi(dw x')): the 1/n factor and the w deapodization
    double dw, xc;      // plane spacing (wavelengths) and the centre x_c of the n - 1 range
    int ncol;           // distinct frequency columns of the extended grid, min(ew, nf)
    int64_t r_stride;   // nk * ew: row-pass buffer per block
};
constexpr int WSORT_MAX = 2048; // records per work item the plane-coordinate sort handles

// w-stacked passes (ivx_wstack.hip).  Plan time: per-block (min, max) partials of the folded w
// (wrange_blocks() pairs per launch), the plane coordinate of every record, the per-work-item
// sort.  Per plane: forward row + column passes into the extended grid; adjoint column + row
// passes accumulating the image gradient into gp.  Per record: residual / data term /
// adjoint coefficients, the model to caller order, caller coefficients to records.
int wrange_blocks();
hipError_t launch_wrange(int64_t n, const int32_t *perm, const real *wsrc, double scale, double *pmin, double *pmax,
                         hipStream_t st);
hipError_t launch_wzeta(int64_t n, const int32_t *perm, const real *wsrc, double scale, double w0, double inv_dw,
                        WZ *out, unsigned int *bad, hipStream_t st);
hipError_t launch_wsort(const WorkItem *work, int n_work, VisCoord *crd, cpx *vis, real *wgt, int32_t *perm, WZ *wz,
                        hipStream_t st);
// the WPlane::cnt table of every work item (after launch_wsort)
hipError_t launch_wcounts(const WorkItem *work, int n_work, const WZ *wz, int ncnt, int32_t *cnt, hipStream_t st);
hipError_t launch_wplane_rows(const Geom &g, const WGeom &wg, int plane, const real *sky, const real *beams,
                              const real *interp, const real *fscale, const real *dq, const cpx *tw, cpx *R,
                              hipStream_t st);
hipError_t launch_wplane_cols(const Geom &g, const WGeom &wg, int plane, const cpx *R, const cpx *tw, cpx *ext,
                              hipStream_t st);
hipError_t launch_wplane_cols_inv(const Geom &g, const WGeom &wg, int plane, const cpx *ext, const cpx *tw, cpx *R,
                                  hipStream_t st);
hipError_t launch_wplane_rows_inv(const Geom &g, const WGeom &wg, int plane, const cpx *R, const real *beams,
                                  const real *fscale, const real *dq, const cpx *tw, real *gp, hipStream_t st);
hipError_t launch_wresid(const WorkItem *work, int n_work, const WGeom &wg, const WZ *wz, const cpx *vis,
                         const real *wgt, cpx *acc, double *jpart, hipStream_t st);
hipError_t launch_wout(const WorkItem *work, int n_work, const WGeom &wg, const WZ *wz, const int32_t *perm,
                       const int64_t *boff, const cpx *acc, cpx *out, hipStream_t st);
hipError_t launch_win(const WorkItem *work, int n_work, const WGeom &wg, const WZ *wz, const int32_t *perm,
                      const int64_t *boff, const real *wgt, bool unweighted, const cpx *in, cpx *q, hipStream_t st);

// w-stacked gridding pass of one plane, mode MODE_WFWD or MODE_WADJ: on the matrix cores
// when variant = GRID_MFMA_VARIANT (float build, windows of at most 16 x 16 cells; occupancy
// as for launch_grid), else the vector gridder (16-lane groups, one visibility per group per
// iteration, nwave waves per work item); prepare_wgrid raises the vector gridder's
// dynamic-LDS limit (call before any stream capture).
hipError_t launch_wgrid(int mode, const Geom &g, const WorkItem *work, int n_work, const VisCoord *crd,
                        const cpx *ext, cpx *slots, const WPlane &wp, int nwave, int variant, int occupancy,
                        hipStream_t st);
hipError_t prepare_wgrid(const Geom &g, int nwave);

// Gridding on the matrix cores (float build, windows of at most 16 x 16 cells, one wave
// per work item): selected by lanes = GRID_MFMA_LANES, variant = GRID_MFMA_VARIANT.
constexpr int GRID_MFMA_LANES = 64;
constexpr int GRID_MFMA_VARIANT = 10 * GRID_MFMA_LANES + 1;
// Register budget of the matrix-core gridder build: waves per SIMD it is compiled for (6 or 7),
// or 0 to choose by the number of work items.
constexpr int GRIDMX_OCC_AUTO = 0;
// Raise the dynamic-LDS limit of the gridding kernels for this geometry (call before any
// stream capture).
// variant = 10 * lanes per visibility (8 or 16) + visibilities per group per iteration (1, 2)
hipError_t prepare_grid(const Geom &g, int nwave, int variant);
// Lane groups per wave of the gridding kernel for kernel width W (one LDS accumulator each).
// lanes = 8 (W <= 8 only) or 16 visibility lanes per group.
int grid_groups_per_wave(int W, int lanes);
// Dynamic LDS of the gridding kernel (bytes); used to pick tiles.
size_t grid_lds_bytes(const Geom &g, int nwave, int lanes);

} // namespace ivx
