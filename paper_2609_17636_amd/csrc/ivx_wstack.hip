// gfx950 kernels of the full forward model (Sect. 2.1, Eq. vis): every pixel carries the factor
// 1/n and the phase w (n - 1), n = sqrt(1 - l^2 - m^2), which the coplanar model drops.
//
// The w dependence is a one-dimensional non-uniform transform along w, done the way the (u, v)
// transform is: with x' = (n - 1) - x_c (x_c the middle of the sub-image's range of n - 1, so
// |x'| <= X / 2) and planes w_p = w0 + p dw, dw = 1 / (sigma_w X),
//   exp(-2 pi i w x') ~= 1 / Phi(dw x') sum_p phi((w - w_p) / dw) exp(-2 pi i w_p x'),
// phi the exponential-of-semicircle kernel over W_w planes and Phi its Fourier transform (the
// same kernel pair and accuracy as the (u, v) gridding at oversampling sigma_w).  Hence
//   V_j = exp(-2 pi i w_j x_c) sum_p phi(zeta_j - p) H_p(u_j, v_j),
//   H_p = the coplanar transform of the complex image f / (n Phi(dw x')) exp(-2 pi i w_p x'),
// with zeta_j = (w_j - w0) / dw.  Each plane is a complex image, so its grid is a full complex
// FFT (no Hermitian half plane): the row and column passes here write the same extended grid
// layout as the coplanar path (rows periodic, columns u - O), filled with the true values at
// negative u, and the vector gridder degrids / spreads each plane with the visibility's w-kernel
// weight (modes MODE_WFWD / MODE_WADJ).  Visibilities keep the coplanar path's Hermitian fold
// (u < 0 -> (-u, -v, -w), conjugate data), valid because the sky is real.
//
//   k_wrange / k_wzeta   plan time: folded w of every record, per-block range, plane coordinate
//   k_wsort              plan time: records of each work item sorted by plane coordinate, so a
//                        plane's visibilities are one contiguous range of the item's list
//   k_wimage_rows        reprojection x beam x flux x deapodization x plane screen, row FFT
//   k_wcol_fwd           column FFT into the extended grid
//   k_wresid             per record: V = exp(-2 pi i w x_c) acc, residual, data term, and the
//                        adjoint coefficient w r exp(+2 pi i w x_c) (in place of acc)
//   k_wcol_inv           alias sum of the folded adjoint grid, inverse column FFT
//   k_wrow_inv           inverse row FFT, conjugate screen, real part, accumulated over planes
//   k_wout / k_win       the forward model to caller order / caller coefficients to records
#include "ivx_internal.hpp"
#include "ivx_fft.hpp"

#include <math.h>

namespace ivx {

namespace {

// exp(-2 pi i t) for t given in cycles (double); the argument is reduced to [-1/2, 1/2] first.
__device__ __forceinline__ cpx unit_phase(double t) {
    const double r = t - rint(t);
#ifdef IVX_REAL_DOUBLE
    double s, c;
    sincospi(2.0 * r, &s, &c);
    return cpx{c, -s};
#else
    float s, c;
    sincospif((float)(2.0 * r), &s, &c);
    return cpx{c, -s};
#endif
}

__device__ __forceinline__ double wz_value(WZ z) {
#ifdef IVX_REAL_DOUBLE
    return z;
#else
    return (double)z * (1.0 / 16777216.0);
#endif
}

constexpr int WR_BLOCKS = 64; // partial (min, max) pairs per block of records

__global__ __launch_bounds__(NT) void k_wrange(int64_t n, const int32_t *__restrict__ perm,
                                               const real *__restrict__ wsrc, double scale,
                                               double *__restrict__ pmin, double *__restrict__ pmax) {
    __shared__ double smin[NT], smax[NT];
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        const int32_t p = perm[i];
        const double w = (double)wsrc[p < 0 ? ~p : p] * scale;
        const double wf = p < 0 ? -w : w;
        lo = fmin(lo, wf);
        hi = fmax(hi, wf);
    }
    smin[threadIdx.x] = lo;
    smax[threadIdx.x] = hi;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        pmin[blockIdx.x] = smin[0];
        pmax[blockIdx.x] = smax[0];
    }
}

// zeta = (w_folded - w0) / dw of one block's records; bad[0] = 1 if one falls outside
// [0, WZ_MAX_PLANES + 1) (or is not finite).
__global__ __launch_bounds__(NT) void k_wzeta(int64_t n, const int32_t *__restrict__ perm,
                                              const real *__restrict__ wsrc, double scale, double w0, double inv_dw,
                                              WZ *__restrict__ out, unsigned int *__restrict__ bad) {
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i >= n) return;
    const int32_t p = perm[i];
    const double w = (double)wsrc[p < 0 ? ~p : p] * scale;
    const double z = ((p < 0 ? -w : w) - w0) * inv_dw;
    if (!(z >= 0.0 && z < (double)(WZ_MAX_PLANES + 1))) {
        atomicOr(bad, 1u);
        out[i] = WZ(0);
        return;
    }
#ifdef IVX_REAL_DOUBLE
    out[i] = z;
#else
    const double q = rint(z * 16777216.0);
    out[i] = q >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)q;
#endif
}

// Permute `words` 32-bit words per record of the n records at `base` by src (LDS staging).
__device__ void permute_words(uint32_t *__restrict__ base, int n, int words, const int16_t *src, uint32_t *stage) {
    for (int w = 0; w < words; ++w) {
        for (int i = threadIdx.x; i < n; i += NT) stage[i] = base[(int64_t)i * words + w];
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += NT) base[(int64_t)i * words + w] = stage[src[i]];
        __syncthreads();
    }
}

__global__ __launch_bounds__(NT) void k_wsort(const WorkItem *__restrict__ work, int n_work, VisCoord *crd, cpx *vis,
                                              real *wgt, int32_t *perm, WZ *wz) {
    __shared__ uint64_t key[WSORT_MAX];
    __shared__ int16_t idx[WSORT_MAX];
    __shared__ uint32_t stage[WSORT_MAX];
    const int64_t wid = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    if (wid >= n_work) return;
    const WorkItem wi = work[wid];
    const int n = wi.count;
    if (n <= 1) return;
    int m = 1;
    while (m < n) m <<= 1;
    WZ *z = wz + wi.begin;
    for (int i = threadIdx.x; i < m; i += NT) {
        if (i < n) {
#ifdef IVX_REAL_DOUBLE
            key[i] = (uint64_t)__double_as_longlong(z[i]); // z >= 0: the bit patterns order as the values
#else
            key[i] = (uint64_t)z[i];
#endif
        } else {
            key[i] = ~0ull;
        }
        idx[i] = (int16_t)i;
    }
    __syncthreads();
    // bitonic sort of (key, index): a total order, so the result is unique
    for (int k = 2; k <= m; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < m; i += NT) {
                const int l = i ^ j;
                if (l > i) {
                    const bool up = (i & k) == 0;
                    const uint64_t ki = key[i], kl = key[l];
                    const int16_t ii = idx[i], il = idx[l];
                    const bool gt = ki > kl || (ki == kl && ii > il);
                    if (gt == up) {
                        key[i] = kl;
                        key[l] = ki;
                        idx[i] = il;
                        idx[l] = ii;
                    }
                }
            }
            __syncthreads();
        }
    }
    permute_words(reinterpret_cast<uint32_t *>(crd + wi.begin), n, (int)(sizeof(VisCoord) / 4), idx, stage);
    permute_words(reinterpret_cast<uint32_t *>(vis + wi.begin), n, (int)(sizeof(cpx) / 4), idx, stage);
    permute_words(reinterpret_cast<uint32_t *>(wgt + wi.begin), n, (int)(sizeof(real) / 4), idx, stage);
    permute_words(reinterpret_cast<uint32_t *>(perm + wi.begin), n, 1, idx, stage);
    permute_words(reinterpret_cast<uint32_t *>(z), n, (int)(sizeof(WZ) / 4), idx, stage);
}

// cnt[wid][h] = records of work item wid with zeta < h / 2 (its records are sorted by zeta):
// one binary search per (work item, h).
__global__ __launch_bounds__(NT) void k_wcounts(const WorkItem *__restrict__ work, int n_work, const WZ *__restrict__ wz,
                                                int ncnt, int32_t *__restrict__ cnt) {
    const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (e >= (int64_t)n_work * ncnt) return;
    const int64_t wid = e / ncnt;
    const int h = (int)(e - wid * ncnt);
    const WorkItem wi = work[wid];
    const WZ *z = wz + wi.begin;
#ifdef IVX_REAL_DOUBLE
    const double key = 0.5 * (double)h;
#else
    const int64_t k = (int64_t)h << 23;
    const uint32_t key = k > (int64_t)0xFFFFFFFFll ? 0xFFFFFFFFu : (uint32_t)k;
#endif
    int lo = 0, hi = wi.count;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (z[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    cnt[e] = lo;
}

// ------------------------------------------------------------------ plane passes
template <int LOGN>
__global__ __launch_bounds__(NT) void k_wimage_rows(Geom g, WGeom wg, int plane, const real *__restrict__ sky,
                                                    const real *__restrict__ beams, const real *__restrict__ interp,
                                                    const real *__restrict__ fscale, const real *__restrict__ dq,
                                                    const cpx *__restrict__ tw, cpx *__restrict__ R) {
    constexpr int N = 1 << LOGN;
    __shared__ cpx buf[N];
    __shared__ cpx tws[tw_len<LOGN>()];
    const int item = blockIdx.y;
    if (plane >= wg.np[item]) return;
    TwStage<LOGN> twr;
    twr.fetch(tw);
    const int tid = threadIdx.x;
    const int k = item / g.C, c = item - (item / g.C) * g.C;
    const int a = blockIdx.x;
    const int nk = g.nk;
    const real *x = sky + (int64_t)c * g.N * g.N;
    const real *A = beams + (int64_t)k * nk * nk;
    const real *G = interp + (int64_t)k * nk * nk * 2;
    const real qa = fscale[c] * dq[a];
    const double w0 = wg.w0[item], pl = (double)plane;
    for (int i = tid; i < N; i += NT) buf[i] = cpx{0, 0};
    __syncthreads();
    for (int b = tid; b < nk; b += NT) {
        const int64_t e = (int64_t)a * nk + b;
        const real f = qa * dq[b] * A[e] * wg.corr[e] * bilinear(x, g.N, G[2 * e], G[2 * e + 1]);
        const cpx s = unit_phase(w0 * wg.xp[e] + pl * wg.tp[e]);
        buf[(b - nk / 2) & (N - 1)] = cpx{f * s.re, f * s.im};
    }
    twr.store(tws);
    __syncthreads();
    fft_lds<LOGN, 1, false>(buf, tws);
    cpx *Ra = R + (int64_t)item * wg.r_stride + (int64_t)a * g.ew;
    for (int ec = tid; ec < g.ew; ec += NT) Ra[ec] = buf[(ec - g.O) & (N - 1)];
}

template <int LOGN, int CB>
__global__ __launch_bounds__(NT) void k_wcol_fwd(Geom g, WGeom wg, int plane, const cpx *__restrict__ R,
                                                 const cpx *__restrict__ tw, cpx *__restrict__ ext) {
    constexpr int N = 1 << LOGN;
    __shared__ cpx buf[CB * N];
    __shared__ cpx tws[tw_len<LOGN>()];
    const int item = blockIdx.y;
    if (plane >= wg.np[item]) return;
    TwStage<LOGN> twr;
    twr.fetch(tw);
    const int tid = threadIdx.x;
    const int c0 = blockIdx.x * CB;
    const int nk = g.nk;
    for (int i = tid; i < CB * N; i += NT) buf[i] = cpx{0, 0};
    __syncthreads();
    const cpx *Ri = R + (int64_t)item * wg.r_stride;
    for (int e = tid; e < nk * CB; e += NT) {
        const int a = e / CB, cc = e - (e / CB) * CB;
        if (c0 + cc < g.ew) buf[((a - nk / 2) & (N - 1)) * CB + cc] = Ri[(int64_t)a * g.ew + c0 + cc];
    }
    twr.store(tws);
    __syncthreads();
    fft_lds<LOGN, CB, false>(buf, tws);
    cpx *E = ext + (int64_t)item * g.ext_stride;
    for (int e = tid; e < CB * g.eh; e += NT) {
        const int cc = e / g.eh, er = e - (e / g.eh) * g.eh;
        if (c0 + cc < g.ew) E[(int64_t)(c0 + cc) * g.eh + er] = buf[((er - g.O) & (N - 1)) * CB + cc];
    }
}

// Adjoint column pass over the ncol = min(ew, N) distinct frequency columns: extended cell
// (er, ec) holds frequency (er - O, ec - O) mod N, so column ec < ncol gathers the extended
// columns ec + m N and, for every frequency row t, the extended rows (t + O) mod N + m N.
template <int LOGN, int CB>
__global__ __launch_bounds__(NT) void k_wcol_inv(Geom g, WGeom wg, int plane, const cpx *__restrict__ ext,
                                                 const cpx *__restrict__ tw, cpx *__restrict__ R) {
    constexpr int N = 1 << LOGN;
    __shared__ cpx buf[CB * N];
    __shared__ cpx tws[tw_len<LOGN>()];
    const int item = blockIdx.y;
    if (plane >= wg.np[item]) return;
    TwStage<LOGN> twr;
    twr.fetch(tw);
    const int tid = threadIdx.x;
    const int c0 = blockIdx.x * CB;
    const int nk = g.nk;
    const cpx *E = ext + (int64_t)item * g.ext_stride;
    for (int e = tid; e < CB * N; e += NT) {
        const int cc = e / N, t = e - (e / N) * N;
        real sr = real(0), si = real(0);
        if (c0 + cc < wg.ncol) {
            for (int ec = c0 + cc; ec < g.ew; ec += N)
                for (int er = (t + g.O) & (N - 1); er < g.eh; er += N) {
                    const cpx h = E[(int64_t)ec * g.eh + er];
                    sr += h.re;
                    si += h.im;
                }
        }
        buf[t * CB + cc] = cpx{sr, si};
    }
    twr.store(tws);
    __syncthreads();
    fft_lds<LOGN, CB, true>(buf, tws);
    cpx *Ri = R + (int64_t)item * wg.r_stride;
    for (int e = tid; e < nk * CB; e += NT) {
        const int a = e / CB, cc = e - (e / CB) * CB;
        if (c0 + cc < wg.ncol) Ri[(int64_t)a * g.ew + c0 + cc] = buf[((a - nk / 2) & (N - 1)) * CB + cc];
    }
}

template <int LOGN>
__global__ __launch_bounds__(NT) void k_wrow_inv(Geom g, WGeom wg, int plane, const cpx *__restrict__ R,
                                                 const real *__restrict__ beams, const real *__restrict__ fscale,
                                                 const real *__restrict__ dq, const cpx *__restrict__ tw,
                                                 real *__restrict__ gp) {
    constexpr int N = 1 << LOGN;
    __shared__ cpx buf[N];
    __shared__ cpx tws[tw_len<LOGN>()];
    const int item = blockIdx.y;
    const int a = blockIdx.x;
    const int nk = g.nk;
    const int tid = threadIdx.x;
    real *out = gp + (int64_t)item * nk * nk + (int64_t)a * nk;
    if (plane >= wg.np[item]) {
        if (plane == 0)
            for (int b = tid; b < nk; b += NT) out[b] = real(0);
        return;
    }
    TwStage<LOGN> twr;
    twr.fetch(tw);
    const int k = item / g.C, c = item - (item / g.C) * g.C;
    for (int i = tid; i < N; i += NT) buf[i] = cpx{0, 0};
    __syncthreads();
    const cpx *Ra = R + (int64_t)item * wg.r_stride + (int64_t)a * g.ew;
    for (int ec = tid; ec < wg.ncol; ec += NT) buf[(ec - g.O) & (N - 1)] = Ra[ec];
    twr.store(tws);
    __syncthreads();
    fft_lds<LOGN, 1, true>(buf, tws);
    const real *A = beams + (int64_t)k * nk * nk;
    const real qa = fscale[c] * dq[a];
    const double w0 = wg.w0[item], pl = (double)plane;
    for (int b = tid; b < nk; b += NT) {
        const int64_t e = (int64_t)a * nk + b;
        const cpx z = buf[(b - nk / 2) & (N - 1)];
        const cpx s = unit_phase(w0 * wg.xp[e] + pl * wg.tp[e]); // the screen; its conjugate applies
        const real v = (z.re * s.re + z.im * s.im) * wg.corr[e] * qa * dq[b] * A[e];
        out[b] = plane == 0 ? v : out[b] + v;
    }
}

// ------------------------------------------------------------- per-record passes
// One 64-lane block per work item.
__device__ __forceinline__ double record_w(const WGeom &wg, int item, WZ z) {
    return wg.w0[item] + wz_value(z) * wg.dw;
}

__global__ __launch_bounds__(64) void k_wresid(const WorkItem *__restrict__ work, int n_work, WGeom wg,
                                               const WZ *__restrict__ wz, const cpx *__restrict__ vis,
                                               const real *__restrict__ wgt, cpx *__restrict__ acc,
                                               double *__restrict__ jpart) {
    const int64_t wid = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    if (wid >= n_work) return;
    const WorkItem wi = work[wid];
    double jsum = 0.0;
    for (int i = threadIdx.x; i < wi.count; i += 64) {
        const int64_t r = wi.begin + i;
        const cpx e = unit_phase(record_w(wg, wi.item, wz[r]) * wg.xc); // exp(-2 pi i w x_c)
        const cpx h = acc[r], y = vis[r];
        const real w = wgt[r];
        const real mr = h.re * e.re - h.im * e.im, mi = h.re * e.im + h.im * e.re;
        const real rr = mr - y.re, ri = mi - y.im;
        jsum += (double)(w * (rr * rr + ri * ri));
        // adjoint coefficient w r exp(+2 pi i w x_c)
        acc[r] = cpx{w * (rr * e.re + ri * e.im), w * (ri * e.re - rr * e.im)};
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) jsum += __shfl_xor(jsum, m, 64);
    if (threadIdx.x == 0) jpart[wid] = 0.5 * jsum;
}

__global__ __launch_bounds__(64) void k_wout(const WorkItem *__restrict__ work, int n_work, WGeom wg,
                                             const WZ *__restrict__ wz, const int32_t *__restrict__ perm,
                                             const int64_t *__restrict__ boff, const cpx *__restrict__ acc,
                                             cpx *__restrict__ out) {
    const int64_t wid = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    if (wid >= n_work) return;
    const WorkItem wi = work[wid];
    cpx *o = out + boff[wi.item];
    for (int i = threadIdx.x; i < wi.count; i += 64) {
        const int64_t r = wi.begin + i;
        const cpx e = unit_phase(record_w(wg, wi.item, wz[r]) * wg.xc);
        const cpx h = acc[r];
        const real mr = h.re * e.re - h.im * e.im, mi = h.re * e.im + h.im * e.re;
        const int32_t p = perm[r];
        if (p < 0) o[~p] = cpx{mr, -mi};
        else o[p] = cpx{mr, mi};
    }
}

__global__ __launch_bounds__(64) void k_win(const WorkItem *__restrict__ work, int n_work, WGeom wg,
                                            const WZ *__restrict__ wz, const int32_t *__restrict__ perm,
                                            const int64_t *__restrict__ boff, const real *__restrict__ wgt,
                                            int unweighted, const cpx *__restrict__ in, cpx *__restrict__ q) {
    const int64_t wid = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    if (wid >= n_work) return;
    const WorkItem wi = work[wid];
    const cpx *src = in + boff[wi.item];
    for (int i = threadIdx.x; i < wi.count; i += 64) {
        const int64_t r = wi.begin + i;
        const cpx e = unit_phase(record_w(wg, wi.item, wz[r]) * wg.xc);
        const int32_t p = perm[r];
        cpx y = src[p < 0 ? ~p : p];
        if (p < 0) y.im = -y.im;
        const real w = unweighted ? real(1) : wgt[r];
        q[r] = cpx{w * (y.re * e.re + y.im * e.im), w * (y.im * e.re - y.re * e.im)};
    }
}

constexpr unsigned WROW = 1u << 22; // work items per grid row (the rest wrap into blockIdx.y)

dim3 work_grid(int n_work) {
    const unsigned gx = (unsigned)n_work < WROW ? (unsigned)n_work : WROW;
    return dim3(gx, (unsigned)((n_work + gx - 1) / gx));
}

template <int LOGN> hipError_t wrows_n(const Geom &g, const WGeom &wg, int plane, const real *sky, const real *beams,
                                       const real *interp, const real *fscale, const real *dq, const cpx *tw, cpx *R,
                                       hipStream_t st) {
    k_wimage_rows<LOGN><<<dim3(g.nk, g.C * g.P), NT, 0, st>>>(g, wg, plane, sky, beams, interp, fscale, dq, tw, R);
    return hipGetLastError();
}

template <int LOGN> hipError_t wcols_n(const Geom &g, const WGeom &wg, int plane, const cpx *R, const cpx *tw,
                                       cpx *ext, hipStream_t st) {
    constexpr int CB = col_batch<LOGN>();
    k_wcol_fwd<LOGN, CB><<<dim3((g.ew + CB - 1) / CB, g.C * g.P), NT, 0, st>>>(g, wg, plane, R, tw, ext);
    return hipGetLastError();
}

template <int LOGN> hipError_t wcols_inv_n(const Geom &g, const WGeom &wg, int plane, const cpx *ext, const cpx *tw,
                                           cpx *R, hipStream_t st) {
    constexpr int CB = col_batch<LOGN>();
    k_wcol_inv<LOGN, CB><<<dim3((wg.ncol + CB - 1) / CB, g.C * g.P), NT, 0, st>>>(g, wg, plane, ext, tw, R);
    return hipGetLastError();
}

template <int LOGN> hipError_t wrows_inv_n(const Geom &g, const WGeom &wg, int plane, const cpx *R, const real *beams,
                                           const real *fscale, const real *dq, const cpx *tw, real *gp,
                                           hipStream_t st) {
    k_wrow_inv<LOGN><<<dim3(g.nk, g.C * g.P), NT, 0, st>>>(g, wg, plane, R, beams, fscale, dq, tw, gp);
    return hipGetLastError();
}

} // namespace

hipError_t launch_wrange(int64_t n, const int32_t *perm, const real *wsrc, double scale, double *pmin, double *pmax,
                         hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_wrange<<<WR_BLOCKS, NT, 0, st>>>(n, perm, wsrc, scale, pmin, pmax);
    return hipGetLastError();
}
int wrange_blocks() { return WR_BLOCKS; }

hipError_t launch_wzeta(int64_t n, const int32_t *perm, const real *wsrc, double scale, double w0, double inv_dw,
                        WZ *out, unsigned int *bad, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_wzeta<<<(unsigned)((n + NT - 1) / NT), NT, 0, st>>>(n, perm, wsrc, scale, w0, inv_dw, out, bad);
    return hipGetLastError();
}

hipError_t launch_wsort(const WorkItem *work, int n_work, VisCoord *crd, cpx *vis, real *wgt, int32_t *perm, WZ *wz,
                        hipStream_t st) {
    if (n_work <= 0) return hipSuccess;
    k_wsort<<<work_grid(n_work), NT, 0, st>>>(work, n_work, crd, vis, wgt, perm, wz);
    return hipGetLastError();
}

hipError_t launch_wcounts(const WorkItem *work, int n_work, const WZ *wz, int ncnt, int32_t *cnt, hipStream_t st) {
    const int64_t tot = (int64_t)n_work * ncnt;
    if (tot <= 0) return hipSuccess;
    k_wcounts<<<(unsigned)((tot + NT - 1) / NT), NT, 0, st>>>(work, n_work, wz, ncnt, cnt);
    return hipGetLastError();
}

#define IVX_LOGN_SWITCH(CALL)                                                                                  \
    switch (g.logn) {                                                                                          \
    case 6: return CALL(6);                                                                                    \
    case 7: return CALL(7);                                                                                    \
    case 8: return CALL(8);                                                                                    \
    case 9: return CALL(9);                                                                                    \
    case 10: return CALL(10);                                                                                  \
    case 11: return CALL(11);                                                                                  \
    default: return hipErrorInvalidValue;                                                                      \
    }

hipError_t launch_wplane_rows(const Geom &g, const WGeom &wg, int plane, const real *sky, const real *beams,
                              const real *interp, const real *fscale, const real *dq, const cpx *tw, cpx *R,
                              hipStream_t st) {
#define IVX_W(L) wrows_n<L>(g, wg, plane, sky, beams, interp, fscale, dq, tw, R, st)
    IVX_LOGN_SWITCH(IVX_W)
#undef IVX_W
}

hipError_t launch_wplane_cols(const Geom &g, const WGeom &wg, int plane, const cpx *R, const cpx *tw, cpx *ext,
                              hipStream_t st) {
#define IVX_W(L) wcols_n<L>(g, wg, plane, R, tw, ext, st)
    IVX_LOGN_SWITCH(IVX_W)
#undef IVX_W
}

hipError_t launch_wplane_cols_inv(const Geom &g, const WGeom &wg, int plane, const cpx *ext, const cpx *tw, cpx *R,
                                  hipStream_t st) {
#define IVX_W(L) wcols_inv_n<L>(g, wg, plane, ext, tw, R, st)
    IVX_LOGN_SWITCH(IVX_W)
#undef IVX_W
}

hipError_t launch_wplane_rows_inv(const Geom &g, const WGeom &wg, int plane, const cpx *R, const real *beams,
                                  const real *fscale, const real *dq, const cpx *tw, real *gp, hipStream_t st) {
#define IVX_W(L) wrows_inv_n<L>(g, wg, plane, R, beams, fscale, dq, tw, gp, st)
    IVX_LOGN_SWITCH(IVX_W)
#undef IVX_W
}
#undef IVX_LOGN_SWITCH

hipError_t launch_wresid(const WorkItem *work, int n_work, const WGeom &wg, const WZ *wz, const cpx *vis,
                         const real *wgt, cpx *acc, double *jpart, hipStream_t st) {
    if (n_work <= 0) return hipSuccess;
    k_wresid<<<work_grid(n_work), 64, 0, st>>>(work, n_work, wg, wz, vis, wgt, acc, jpart);
    return hipGetLastError();
}

hipError_t launch_wout(const WorkItem *work, int n_work, const WGeom &wg, const WZ *wz, const int32_t *perm,
                       const int64_t *boff, const cpx *acc, cpx *out, hipStream_t st) {
    if (n_work <= 0) return hipSuccess;
    k_wout<<<work_grid(n_work), 64, 0, st>>>(work, n_work, wg, wz, perm, boff, acc, out);
    return hipGetLastError();
}

hipError_t launch_win(const WorkItem *work, int n_work, const WGeom &wg, const WZ *wz, const int32_t *perm,
                      const int64_t *boff, const real *wgt, bool unweighted, const cpx *in, cpx *q, hipStream_t st) {
    if (n_work <= 0) return hipSuccess;
    k_win<<<work_grid(n_work), 64, 0, st>>>(work, n_work, wg, wz, perm, boff, wgt, unweighted ? 1 : 0, in, q);
    return hipGetLastError();
}

} // namespace ivx
