/*
 * FP64 direct (non-uniform) discrete Fourier transform of one primary-beam-weighted
 * sub-image, and its explicit adjoint.  TEST INFRASTRUCTURE ONLY: this file is the
 * oracle that the HIP path is checked against; no product code may link or call it.
 *
 * Coplanar forward model (Sect. 2.1, the small-angle form of Eq. vis):
 *     V_j = sum_{a,b} f[a][b] * exp(-2 pi i (u_j l_b + v_j m_a)),
 *     l_b = (b - n/2) * delta,   m_a = (a - n/2) * delta,
 * with l along columns (b) and m along rows (a).  f is the real sub-image already
 * multiplied by the primary beam and the flux scale.
 *
 * Because (b - n/2) and (a - n/2) are integers, exp(-2 pi i u_j delta (b - n/2)) only
 * depends on the fractional part of u_j * delta; the phase is formed from
 * frac(u_j * delta) so that large |u| keeps full FP64 precision.  The exponential of a
 * sum is evaluated as the product of the two factors, each from its own sin/cos call
 * (no recurrences).
 *
 * Adjoint (gradient of a real-sky least-squares term, Sect. 2.2):
 *     g[a][b] = Re sum_j c_j * exp(+2 pi i (u_j l_b + v_j m_a)).
 *
 * Parallel over visibilities with OpenMP; the adjoint keeps one private image per
 * thread and adds them in thread order, so results do not depend on scheduling.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

static double frac_part(double t) { return t - floor(t); }

int orc_num_threads(void) { return omp_get_max_threads(); }

/* f: [n][n] row-major; uv: [m][2] (u, v) in wavelengths; out: [m][2] (re, im). */
void orc_dft_forward(int n, double delta, const double *f, int64_t m, const double *uv,
                     double *out)
{
    const int c = n / 2;
    #pragma omp parallel
    {
        double *cb = (double *)malloc(sizeof(double) * n);
        double *sb = (double *)malloc(sizeof(double) * n);
        double *ca = (double *)malloc(sizeof(double) * n);
        double *sa = (double *)malloc(sizeof(double) * n);
        #pragma omp for schedule(static)
        for (int64_t j = 0; j < m; ++j) {
            const double fu = frac_part(uv[2 * j] * delta);
            const double fv = frac_part(uv[2 * j + 1] * delta);
            for (int b = 0; b < n; ++b) {
                const double th = 2.0 * M_PI * fu * (double)(b - c);
                cb[b] = cos(th);
                sb[b] = sin(th);
            }
            for (int a = 0; a < n; ++a) {
                const double th = 2.0 * M_PI * fv * (double)(a - c);
                ca[a] = cos(th);
                sa[a] = sin(th);
            }
            double vr = 0.0, vi = 0.0;
            for (int a = 0; a < n; ++a) {
                /* row sum  S_a = sum_b f[a][b] exp(-i th_b) */
                double sr = 0.0, si = 0.0;
                const double *row = f + (int64_t)a * n;
                for (int b = 0; b < n; ++b) {
                    sr += row[b] * cb[b];
                    si -= row[b] * sb[b];
                }
                /* times exp(-i th_a) = ca - i sa */
                vr += sr * ca[a] + si * sa[a];
                vi += si * ca[a] - sr * sa[a];
            }
            out[2 * j] = vr;
            out[2 * j + 1] = vi;
        }
        free(cb); free(sb); free(ca); free(sa);
    }
}

/* coef: [m][2] complex weights c_j; g: [n][n] output (overwritten). */
void orc_dft_adjoint(int n, double delta, int64_t m, const double *uv, const double *coef,
                     double *g)
{
    const int c = n / 2;
    const int nt = omp_get_max_threads();
    double *acc = (double *)calloc((size_t)nt * n * n, sizeof(double));
    #pragma omp parallel num_threads(nt)
    {
        const int t = omp_get_thread_num();
        double *mine = acc + (size_t)t * n * n;
        double *cb = (double *)malloc(sizeof(double) * n);
        double *sb = (double *)malloc(sizeof(double) * n);
        #pragma omp for schedule(static)
        for (int64_t j = 0; j < m; ++j) {
            const double fu = frac_part(uv[2 * j] * delta);
            const double fv = frac_part(uv[2 * j + 1] * delta);
            const double cr = coef[2 * j], ci = coef[2 * j + 1];
            for (int b = 0; b < n; ++b) {
                const double th = 2.0 * M_PI * fu * (double)(b - c);
                cb[b] = cos(th);
                sb[b] = sin(th);
            }
            for (int a = 0; a < n; ++a) {
                const double th = 2.0 * M_PI * fv * (double)(a - c);
                /* t = c_j * exp(+i th_a) */
                const double tr = cr * cos(th) - ci * sin(th);
                const double ti = cr * sin(th) + ci * cos(th);
                double *row = mine + (size_t)a * n;
                /* Re(t * exp(+i th_b)) */
                for (int b = 0; b < n; ++b) row[b] += tr * cb[b] - ti * sb[b];
            }
        }
        free(cb); free(sb);
    }
    memset(g, 0, sizeof(double) * n * n);
    for (int t = 0; t < nt; ++t) {
        const double *mine = acc + (size_t)t * n * n;
        for (int64_t i = 0; i < (int64_t)n * n; ++i) g[i] += mine[i];
    }
    free(acc);
}

/* The adjoint evaluated at selected pixels only (one direct sum over all visibilities per
 * pixel), for sampled checks at sizes where the full adjoint image is too slow.
 * pix: [np][2] (a, b); out: [np]. */
void orc_dft_adjoint_pixels(int n, double delta, int64_t m, const double *uv, const double *coef,
                            int64_t np, const int32_t *pix, double *out)
{
    const int c = n / 2;
    #pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < np; ++q) {
        const int a = pix[2 * q], b = pix[2 * q + 1];
        double s = 0.0;
        for (int64_t j = 0; j < m; ++j) {
            const double fu = frac_part(uv[2 * j] * delta);
            const double fv = frac_part(uv[2 * j + 1] * delta);
            const double th = 2.0 * M_PI * (fu * (double)(b - c) + fv * (double)(a - c));
            s += coef[2 * j] * cos(th) - coef[2 * j + 1] * sin(th);
        }
        out[q] = s;
    }
}

/*
 * Full forward model with the non-coplanar term (Sect. 2.1, Eq. vis): every pixel carries
 * the factor 1/n and the phase w (n - 1), where n = sqrt(1 - l^2 - m^2) is the third
 * direction cosine of pixel (a, b):
 *     V_j = sum_{a,b} f[a][b] / n_ab * exp(-2 pi i (u_j l_b + v_j m_a + w_j (n_ab - 1))).
 * n - 1 is formed as -(l^2 + m^2) / (1 + n), the same number without the cancellation of
 * sqrt(.) - 1 near the phase centre.  The (u, v) factors are formed as in the coplanar
 * model; the w factor takes one sin/cos pair per visibility and pixel.  Pixels need
 * l^2 + m^2 < 1 (the caller checks).
 *
 * uvw: [m][3] (u, v, w) in wavelengths.
 */
static void pixel_n(int n, double delta, double *inv_n, double *nm1)
{
    const int c = n / 2;
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
            const double l = (double)(b - c) * delta, mm = (double)(a - c) * delta;
            const double r2 = l * l + mm * mm;
            const double nn = sqrt(1.0 - r2);
            inv_n[a * n + b] = 1.0 / nn;
            nm1[a * n + b] = -r2 / (1.0 + nn);
        }
}

void orc_dft_forward_w(int n, double delta, const double *f, int64_t m, const double *uvw,
                       double *out)
{
    const int c = n / 2;
    double *inv_n = (double *)malloc(sizeof(double) * n * n);
    double *nm1 = (double *)malloc(sizeof(double) * n * n);
    pixel_n(n, delta, inv_n, nm1);
    #pragma omp parallel
    {
        double *cb = (double *)malloc(sizeof(double) * n);
        double *sb = (double *)malloc(sizeof(double) * n);
        #pragma omp for schedule(static)
        for (int64_t j = 0; j < m; ++j) {
            const double fu = frac_part(uvw[3 * j] * delta);
            const double fv = frac_part(uvw[3 * j + 1] * delta);
            const double w = uvw[3 * j + 2];
            for (int b = 0; b < n; ++b) {
                const double th = 2.0 * M_PI * fu * (double)(b - c);
                cb[b] = cos(th);
                sb[b] = sin(th);
            }
            double vr = 0.0, vi = 0.0;
            for (int a = 0; a < n; ++a) {
                const double tha = 2.0 * M_PI * fv * (double)(a - c);
                const double ca = cos(tha), sa = sin(tha);
                /* row sum  S_a = sum_b (f / n) exp(-i (th_b + 2 pi w (n - 1))) */
                double sr = 0.0, si = 0.0;
                for (int b = 0; b < n; ++b) {
                    const int64_t q = (int64_t)a * n + b;
                    const double thw = 2.0 * M_PI * w * nm1[q];
                    const double cw = cos(thw), sw = sin(thw);
                    /* exp(-i th_b) exp(-i thw) = (cb - i sb)(cw - i sw) */
                    const double er = cb[b] * cw - sb[b] * sw;
                    const double ei = -(sb[b] * cw + cb[b] * sw);
                    const double fv_ = f[q] * inv_n[q];
                    sr += fv_ * er;
                    si += fv_ * ei;
                }
                /* times exp(-i th_a) = ca - i sa */
                vr += sr * ca + si * sa;
                vi += si * ca - sr * sa;
            }
            out[2 * j] = vr;
            out[2 * j + 1] = vi;
        }
        free(cb); free(sb);
    }
    free(inv_n); free(nm1);
}

/* Adjoint of orc_dft_forward_w as a map from real images:
 *     g[a][b] = Re sum_j c_j / n_ab * exp(+2 pi i (u_j l_b + v_j m_a + w_j (n_ab - 1))). */
void orc_dft_adjoint_w(int n, double delta, int64_t m, const double *uvw, const double *coef,
                       double *g)
{
    const int c = n / 2;
    const int nt = omp_get_max_threads();
    double *inv_n = (double *)malloc(sizeof(double) * n * n);
    double *nm1 = (double *)malloc(sizeof(double) * n * n);
    pixel_n(n, delta, inv_n, nm1);
    double *acc = (double *)calloc((size_t)nt * n * n, sizeof(double));
    #pragma omp parallel num_threads(nt)
    {
        const int t = omp_get_thread_num();
        double *mine = acc + (size_t)t * n * n;
        double *cb = (double *)malloc(sizeof(double) * n);
        double *sb = (double *)malloc(sizeof(double) * n);
        #pragma omp for schedule(static)
        for (int64_t j = 0; j < m; ++j) {
            const double fu = frac_part(uvw[3 * j] * delta);
            const double fv = frac_part(uvw[3 * j + 1] * delta);
            const double w = uvw[3 * j + 2];
            const double cr = coef[2 * j], ci = coef[2 * j + 1];
            for (int b = 0; b < n; ++b) {
                const double th = 2.0 * M_PI * fu * (double)(b - c);
                cb[b] = cos(th);
                sb[b] = sin(th);
            }
            for (int a = 0; a < n; ++a) {
                const double th = 2.0 * M_PI * fv * (double)(a - c);
                /* t = c_j * exp(+i th_a) */
                const double tr = cr * cos(th) - ci * sin(th);
                const double ti = cr * sin(th) + ci * cos(th);
                double *row = mine + (size_t)a * n;
                for (int b = 0; b < n; ++b) {
                    const int64_t q = (int64_t)a * n + b;
                    const double thw = 2.0 * M_PI * w * nm1[q];
                    /* exp(+i th_b) exp(+i thw) */
                    const double er = cb[b] * cos(thw) - sb[b] * sin(thw);
                    const double ei = sb[b] * cos(thw) + cb[b] * sin(thw);
                    row[b] += (tr * er - ti * ei) * inv_n[q];
                }
            }
        }
        free(cb); free(sb);
    }
    memset(g, 0, sizeof(double) * n * n);
    for (int t = 0; t < nt; ++t) {
        const double *mine = acc + (size_t)t * n * n;
        for (int64_t i = 0; i < (int64_t)n * n; ++i) g[i] += mine[i];
    }
    free(acc); free(inv_n); free(nm1);
}

/* orc_dft_adjoint_w at selected pixels only (one direct sum per pixel). */
void orc_dft_adjoint_w_pixels(int n, double delta, int64_t m, const double *uvw, const double *coef,
                              int64_t np, const int32_t *pix, double *out)
{
    const int c = n / 2;
    #pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < np; ++q) {
        const int a = pix[2 * q], b = pix[2 * q + 1];
        const double l = (double)(b - c) * delta, mm = (double)(a - c) * delta;
        const double r2 = l * l + mm * mm;
        const double nn = sqrt(1.0 - r2);
        const double nm1 = -r2 / (1.0 + nn);
        double s = 0.0;
        for (int64_t j = 0; j < m; ++j) {
            const double fu = frac_part(uvw[3 * j] * delta);
            const double fv = frac_part(uvw[3 * j + 1] * delta);
            const double th = 2.0 * M_PI * (fu * (double)(b - c) + fv * (double)(a - c) + uvw[3 * j + 2] * nm1);
            s += coef[2 * j] * cos(th) - coef[2 * j + 1] * sin(th);
        }
        out[q] = s / nn;
    }
}
