// The data processor of the paper's pipeline on the GPU (Sect. 3.3): SIN interpolation grids
// of every pointing, their inverse for the deprojection of Sect. 4.4.1 (Eq. sin_deprojection),
// primary beams resampled to the sky pixel scale, linear mosaicking (Eq. linear, Eq. pb_eff)
// and the C-ABI side of feathering (App. B; its FFT kernels live with the other FFTs).
//
// The orthographic (SIN) projection about a tangent point (ra0, dec0), in its trigonometric
// form (Calabretta & Greisen 2002):
//   l = cos dec sin(ra - ra0)
//   m = sin dec cos dec0 - cos dec sin dec0 cos(ra - ra0)
//   n = sin dec sin dec0 + cos dec cos dec0 cos(ra - ra0)
// and its inverse on the near hemisphere, n = sqrt(1 - l^2 - m^2):
//   dec = asin(m cos dec0 + n sin dec0),  ra = ra0 + atan2(l, n cos dec0 - m sin dec0).
// All coordinate arithmetic is FP64.
#include "ivx_internal.hpp"
#include "ivx_dataproc.h"

#include <math.h>

#include <cmath>
#include <string>

namespace ivx {
ivx_status set_error(ivx_status s, const std::string &msg); // shared thread-local message
hipError_t launch_feather(int n_chan, int n, double delta, double theta, const real *interf, const real *sd, real *out,
                          void *work, hipStream_t st);
int64_t feather_work_bytes(int n_chan, int n);
} // namespace ivx

namespace {

using namespace ivx;

constexpr int BT = 256;
constexpr double FAR_SIDE = -1e9; // deprojection of a direction behind the tangent point

struct Tangent {
    double ra, sd, cd; // ra0, sin dec0, cos dec0
};

__host__ __device__ inline Tangent tangent(double ra, double dec) { return Tangent{ra, sin(dec), cos(dec)}; }

// direction cosines of (ra, dec) about t
__device__ inline void sin_project(const Tangent &t, double ra, double dec, double &l, double &m, double &n) {
    double sa, ca, sdc, cdc;
    sincos(ra - t.ra, &sa, &ca);
    sincos(dec, &sdc, &cdc);
    l = cdc * sa;
    m = sdc * t.cd - cdc * t.sd * ca;
    n = sdc * t.sd + cdc * t.cd * ca;
}

// (ra, dec) of (l, m) on the near hemisphere of t
__device__ inline void sin_unproject(const Tangent &t, double l, double m, double &ra, double &dec) {
    const double q = 1.0 - l * l - m * m;
    const double n = sqrt(q > 0.0 ? q : 0.0);
    dec = asin(fmin(1.0, fmax(-1.0, m * t.cd + n * t.sd)));
    ra = t.ra + atan2(l, n * t.cd - m * t.sd);
}

// grids[a][b] = sky-frame (row, col) of sub-pixel (a, b) of the pointing tangent at tk
__global__ __launch_bounds__(BT) void k_sin_grid(int n_sky, double sky_delta, Tangent tsky, int n_sub, double sub_delta,
                                                 Tangent tk, real *__restrict__ grid) {
    const int64_t e = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (e >= (int64_t)n_sub * n_sub) return;
    const int a = (int)(e / n_sub), b = (int)(e - (int64_t)a * n_sub);
    double ra, dec, l, m, n;
    sin_unproject(tk, (b - n_sub / 2) * sub_delta, (a - n_sub / 2) * sub_delta, ra, dec);
    sin_project(tsky, ra, dec, l, m, n);
    grid[2 * e] = (real)(m / sky_delta + n_sky / 2);
    grid[2 * e + 1] = (real)(l / sky_delta + n_sky / 2);
}

// grids[i][j] = (row, col) in the sub-image of the pointing tangent at tk of sky pixel (i, j)
__global__ __launch_bounds__(BT) void k_deproj_grid(int n_sky, double sky_delta, Tangent tsky, int n_sub,
                                                    double sub_delta, Tangent tk, real *__restrict__ grid) {
    const int64_t e = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (e >= (int64_t)n_sky * n_sky) return;
    const int i = (int)(e / n_sky), j = (int)(e - (int64_t)i * n_sky);
    double ra, dec, l, m, n;
    sin_unproject(tsky, (j - n_sky / 2) * sky_delta, (i - n_sky / 2) * sky_delta, ra, dec);
    sin_project(tk, ra, dec, l, m, n);
    const bool near = n > 0.0;
    grid[2 * e] = (real)(near ? m / sub_delta + n_sub / 2 : FAR_SIDE);
    grid[2 * e + 1] = (real)(near ? l / sub_delta + n_sub / 2 : FAR_SIDE);
}

// bilinear sample of an h x w image at (row, col); pixel (i, j) sits at (i, j); 0 outside
__device__ inline real sample(const real *__restrict__ img, int h, int w, real row, real col) {
    if (!(row > real(-1) && row < real(h) && col > real(-1) && col < real(w))) return real(0);
    const real fr = floor(row), fc = floor(col);
    const int i0 = (int)fr, j0 = (int)fc;
    const real fy = row - fr, fx = col - fc;
    const bool r0 = i0 >= 0, r1 = i0 + 1 < h, c0 = j0 >= 0, c1 = j0 + 1 < w;
    const real *p = img + (int64_t)i0 * w + j0;
    const real v00 = (r0 && c0) ? p[0] : real(0), v01 = (r0 && c1) ? p[1] : real(0);
    const real v10 = (r1 && c0) ? p[w] : real(0), v11 = (r1 && c1) ? p[w + 1] : real(0);
    return (real(1) - fy) * ((real(1) - fx) * v00 + fx * v01) + fy * ((real(1) - fx) * v10 + fx * v11);
}

__global__ __launch_bounds__(BT) void k_resample_beam(const real *__restrict__ in, int nb, double beam_delta,
                                                      int n_sub, double sub_delta, real *__restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * BT + threadIdx.x;
    const int k = blockIdx.y;
    if (e >= (int64_t)n_sub * n_sub) return;
    const int a = (int)(e / n_sub), b = (int)(e - (int64_t)a * n_sub);
    const double ratio = sub_delta / beam_delta;
    const real row = (real)((a - n_sub / 2) * ratio + nb / 2), col = (real)((b - n_sub / 2) * ratio + nb / 2);
    out[(int64_t)k * n_sub * n_sub + e] = sample(in + (int64_t)k * nb * nb, nb, nb, row, col);
}

// One thread per (sky pixel, group of MOS_CG channels): per pointing the deprojected position,
// the bilinear taps and the beam weight are formed once and applied to every channel of the
// group (the per-channel sums run over the pointings in index order, as before).
constexpr int MOS_CG = 16;
__global__ __launch_bounds__(BT) void k_linear_mosaic(int P, int C, int n_sub, const real *__restrict__ sub,
                                                      const real *__restrict__ beams, int N,
                                                      const real *__restrict__ deproj, real pb_min2,
                                                      real *__restrict__ image, real *__restrict__ pb_eff) {
    const int64_t r = (int64_t)blockIdx.x * BT + threadIdx.x;
    const int64_t NN = (int64_t)N * N;
    if (r >= NN) return;
    const int c0 = blockIdx.y * MOS_CG;
    const int cn = min(MOS_CG, C - c0);
    const int64_t n2 = (int64_t)n_sub * n_sub;
    real num[MOS_CG];
#pragma unroll
    for (int q = 0; q < MOS_CG; ++q) num[q] = real(0);
    real den = real(0);
    for (int k = 0; k < P; ++k) {
        const real row = deproj[((int64_t)k * NN + r) * 2], col = deproj[((int64_t)k * NN + r) * 2 + 1];
        if (!(row > real(-1) && row < real(n_sub) && col > real(-1) && col < real(n_sub))) continue;
        const real fr = floor(row), fc = floor(col);
        const int i0 = (int)fr, j0 = (int)fc;
        const real fy = row - fr, fx = col - fc;
        const bool r0 = i0 >= 0, r1 = i0 + 1 < n_sub, q0 = j0 >= 0, q1 = j0 + 1 < n_sub;
        const real w00 = (r0 && q0) ? (real(1) - fy) * (real(1) - fx) : real(0);
        const real w01 = (r0 && q1) ? (real(1) - fy) * fx : real(0);
        const real w10 = (r1 && q0) ? fy * (real(1) - fx) : real(0);
        const real w11 = (r1 && q1) ? fy * fx : real(0);
        // clamped tap offsets: a weight is zero wherever its tap is outside
        const int64_t o00 = (int64_t)max(i0, 0) * n_sub + max(j0, 0);
        const int64_t o01 = (int64_t)max(i0, 0) * n_sub + min(j0 + 1, n_sub - 1);
        const int64_t o10 = (int64_t)min(i0 + 1, n_sub - 1) * n_sub + max(j0, 0);
        const int64_t o11 = (int64_t)min(i0 + 1, n_sub - 1) * n_sub + min(j0 + 1, n_sub - 1);
        auto tap = [&](const real *img) {
            return (real(1) - fy) * ((real(1) - fx) * (w00 != real(0) ? img[o00] : real(0)) +
                                      fx * (w01 != real(0) ? img[o01] : real(0))) +
                   fy * ((real(1) - fx) * (w10 != real(0) ? img[o10] : real(0)) +
                         fx * (w11 != real(0) ? img[o11] : real(0)));
        };
        const real A = tap(beams + (int64_t)k * n2);
        if (A == real(0)) continue;
        const real A2 = A * A;
        const real *sk = sub + ((int64_t)k * C + c0) * n2;
#pragma unroll
        for (int q = 0; q < MOS_CG; ++q)
            if (q < cn) num[q] += A2 * tap(sk + (int64_t)q * n2);
        den += A2;
    }
    const bool keep = den > real(0) && den >= pb_min2;
#pragma unroll
    for (int q = 0; q < MOS_CG; ++q)
        if (q < cn) image[(int64_t)(c0 + q) * NN + r] = keep ? num[q] / den : real(0);
    if (pb_eff && blockIdx.y == 0) pb_eff[r] = sqrt(den);
}

unsigned blocks(int64_t n) { return (unsigned)((n + BT - 1) / BT); }

ivx_status check_frame(const ivx_sin_frame *f) {
    if (!f || f->n < 4 || !(f->delta > 0.0) || !std::isfinite(f->ra) || !std::isfinite(f->dec) || f->reserved != 0)
        return set_error(IVX_EINVAL, "bad sky frame (n >= 4, delta > 0, finite tangent point, reserved 0)");
    return IVX_OK;
}

ivx_status hip_status(hipError_t e, const char *what) {
    if (e == hipSuccess) return IVX_OK;
    return set_error(IVX_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

} // namespace

extern "C" {

ivx_status ivx_dp_sin_grids(const ivx_sin_frame *sky, int32_t n_point, const double *centres, int32_t n_sub,
                            double sub_delta, ivx_real *grids, void *stream) {
    ivx_status s = check_frame(sky);
    if (s != IVX_OK) return s;
    if (n_point < 1 || !centres || !grids || n_sub < 4 || !(sub_delta > 0.0))
        return set_error(IVX_EINVAL, "bad ivx_dp_sin_grids arguments");
    const Tangent ts = tangent(sky->ra, sky->dec);
    const int64_t n2 = (int64_t)n_sub * n_sub;
    for (int k = 0; k < n_point; ++k) {
        if (!std::isfinite(centres[2 * k]) || !std::isfinite(centres[2 * k + 1]))
            return set_error(IVX_EINVAL, "pointing centres must be finite");
        k_sin_grid<<<blocks(n2), BT, 0, (hipStream_t)stream>>>(sky->n, sky->delta, ts, n_sub, sub_delta,
                                                               tangent(centres[2 * k], centres[2 * k + 1]),
                                                               grids + (int64_t)k * n2 * 2);
    }
    return hip_status(hipGetLastError(), "k_sin_grid");
}

ivx_status ivx_dp_deprojection_grids(const ivx_sin_frame *sky, int32_t n_point, const double *centres,
                                     int32_t n_sub, double sub_delta, ivx_real *grids, void *stream) {
    ivx_status s = check_frame(sky);
    if (s != IVX_OK) return s;
    if (n_point < 1 || !centres || !grids || n_sub < 4 || !(sub_delta > 0.0))
        return set_error(IVX_EINVAL, "bad ivx_dp_deprojection_grids arguments");
    const Tangent ts = tangent(sky->ra, sky->dec);
    const int64_t nn = (int64_t)sky->n * sky->n;
    for (int k = 0; k < n_point; ++k) {
        if (!std::isfinite(centres[2 * k]) || !std::isfinite(centres[2 * k + 1]))
            return set_error(IVX_EINVAL, "pointing centres must be finite");
        k_deproj_grid<<<blocks(nn), BT, 0, (hipStream_t)stream>>>(sky->n, sky->delta, ts, n_sub, sub_delta,
                                                                  tangent(centres[2 * k], centres[2 * k + 1]),
                                                                  grids + (int64_t)k * nn * 2);
    }
    return hip_status(hipGetLastError(), "k_deproj_grid");
}

ivx_status ivx_dp_resample_beams(int32_t n_point, const ivx_real *beams_in, int32_t nb, double beam_delta,
                                 int32_t n_sub, double sub_delta, ivx_real *beams_out, void *stream) {
    if (n_point < 1 || n_point > 65535 || !beams_in || !beams_out || nb < 2 || n_sub < 4 || !(beam_delta > 0.0) ||
        !(sub_delta > 0.0))
        return set_error(IVX_EINVAL, "bad ivx_dp_resample_beams arguments");
    const int64_t n2 = (int64_t)n_sub * n_sub;
    k_resample_beam<<<dim3(blocks(n2), n_point), BT, 0, (hipStream_t)stream>>>(beams_in, nb, beam_delta, n_sub,
                                                                               sub_delta, beams_out);
    return hip_status(hipGetLastError(), "k_resample_beam");
}

ivx_status ivx_linear_mosaic(int32_t n_point, int32_t n_chan, int32_t n_sub, const ivx_real *sub_images,
                             const ivx_real *beams, int32_t n_sky, const ivx_real *deproj, double pb_min,
                             ivx_real *image, ivx_real *pb_eff, void *stream) {
    if (n_point < 1 || n_chan < 1 || n_sub < 4 || n_sky < 4 || !sub_images || !beams || !deproj || !image ||
        !(pb_min >= 0.0) || !std::isfinite(pb_min))
        return set_error(IVX_EINVAL, "bad ivx_linear_mosaic arguments");
    const dim3 grid(blocks((int64_t)n_sky * n_sky), (unsigned)((n_chan + MOS_CG - 1) / MOS_CG));
    k_linear_mosaic<<<grid, BT, 0, (hipStream_t)stream>>>(n_point, n_chan, n_sub, sub_images, beams, n_sky, deproj,
                                                          (real)(pb_min * pb_min), image, pb_eff);
    return hip_status(hipGetLastError(), "k_linear_mosaic");
}

int64_t ivx_feather_work_bytes(int32_t n_chan, int32_t n) {
    if (n_chan < 1 || n < 64 || n > 2048 || (n & (n - 1))) return -1;
    return feather_work_bytes(n_chan, n);
}

ivx_status ivx_feather(int32_t n_chan, int32_t n, double delta, double theta, const ivx_real *interf,
                       const ivx_real *single_dish, ivx_real *out, void *work, void *stream) {
    if (n_chan < 1 || n < 64 || n > 2048 || (n & (n - 1)) || !(delta > 0.0) || !(theta >= 0.0) ||
        !std::isfinite(theta) || !interf || !single_dish || !out || !work)
        return set_error(IVX_EINVAL, "bad ivx_feather arguments (n a power of two in [64, 2048])");
    return hip_status(launch_feather(n_chan, n, delta, theta, interf, single_dish, out, work, (hipStream_t)stream),
                      "feather");
}

} // extern "C"
