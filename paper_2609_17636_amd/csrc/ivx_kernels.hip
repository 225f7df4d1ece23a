// gfx950 kernels of one Classic3D objective/gradient evaluation.
//
// Forward direction (Sect. 2.1), per (pointing k, channel c) block:
//   k_image_rows  bilinear SIN reprojection of the sky (Eq. sin_projection) x beam x flux
//                 scale x deapodization, zero-padded to the fine grid, and the row FFT of
//                 two real rows packed in one complex transform (half spectrum kept);
//   k_col_fwd     column FFT of the n_sub non-zero rows, written to an extended grid that
//                 carries the periodic wrap in rows and the Hermitian mirror in columns,
//                 so a footprint never needs a modulo;
//   k_gridmx /    per fine-grid tile: interpolate every visibility from the grid window
//   k_grid        (degridding), form the residual and its weighted square (Sect. 2.2,
//                 J_k), and spread w * r back into the window's accumulation (matrix-core
//                 products in registers, or per-wave LDS accumulators; no global atomics);
//                 the window is written to a private slot.
// Adjoint direction (gradient, Sect. 3.4):
//   k_ext_sum     sum the slots covering each cell of the extended grid (the fold);
//   k_col_inv     alias sum and symmetrisation H -> (H + conj H(-t))/2 as it loads, which
//                 makes the real part of the adjoint a half-spectrum inverse FFT; inverse
//                 column FFT, keeping the n_sub rows of the sub-image;
//   k_row_inv     inverse row FFT of two rows at once, crop, deapodization x beam x flux;
//   k_sky         transpose of the bilinear reprojection (gather over a pixel-major CSR,
//                 fixed order), plus the Laplacian regulariser (Eq. 3) and the single-dish
//                 gradient (Sect. 2.4); k_sd_rows / k_sd_cols give the single-dish model.
// The NUFFT is the exponential-of-semicircle scheme of Barnett et al. (2019): kernel
// phi(z) = exp(beta (sqrt(1 - (2z/W)^2) - 1)), deapodization by its Fourier transform.
#include "ivx_internal.hpp"
#include "ivx_fft.hpp"

#include <math.h>

#include <algorithm>

#include <type_traits>

namespace ivx {

// --------------------------------------------------------------- forward row pass
template <int LOGN>
__global__ __launch_bounds__(NT) void k_image_rows(Geom g, const real *__restrict__ sky,
                                                   const real *__restrict__ beams,
                                                   const real *__restrict__ interp,
                                                   const real *__restrict__ fscale,
                                                   const real *__restrict__ dq,
                                                   const cpx *__restrict__ tw, cpx *__restrict__ R) {
    constexpr int N = 1 << LOGN;
    __shared__ cpx buf[N + 1]; // + a sink cell for the stores of positions past the end
    __shared__ cpx tws[tw_len<LOGN>()];
    TwStage<LOGN> twr;
    twr.fetch(tw);
    const int tid = threadIdx.x;
    const int item = blockIdx.y;
    const int k = item / g.C, c = item - (item / g.C) * g.C;
    const int a0 = 2 * blockIdx.x;
    const int nk = g.nk;
    const real *x = sky + (int64_t)c * g.N * g.N;
    const real *A = beams + (int64_t)k * nk * nk;
    const real *G = interp + (int64_t)k * nk * nk * 2;
    const real s = fscale[c];
    for (int i = tid; i < N; i += NT) buf[i] = cpx{0, 0};
    __syncthreads();
    const real q0 = s * dq[a0], q1 = s * dq[a0 + 1];
    // IR_U columns per thread: their beam values and sample positions are requested together,
    // then every sky tap of both rows (positions past the end read column 0 and store to the
    // sink cell): two round trips instead of two per row and column
    constexpr int IR_U = 2;
    for (int b0 = tid; b0 < nk; b0 += IR_U * NT) {
        real dv[IR_U], a_0[IR_U], a_1[IR_U], y0[IR_U], x0[IR_U], y1[IR_U], x1[IR_U];
#pragma unroll
        for (int u = 0; u < IR_U; ++u) {
            const int b = b0 + u * NT < nk ? b0 + u * NT : 0;
            const int64_t e0 = (int64_t)a0 * nk + b, e1 = e0 + nk;
            dv[u] = dq[b];
            a_0[u] = A[e0];
            a_1[u] = A[e1];
            y0[u] = G[2 * e0];
            x0[u] = G[2 * e0 + 1];
            y1[u] = G[2 * e1];
            x1[u] = G[2 * e1 + 1];
        }
        BilinearTaps t0[IR_U], t1[IR_U];
        real p0[IR_U][4], p1[IR_U][4];
#pragma unroll
        for (int u = 0; u < IR_U; ++u) {
            t0[u] = bilinear_taps(g.N, y0[u], x0[u]);
            t1[u] = bilinear_taps(g.N, y1[u], x1[u]);
        }
#pragma unroll
        for (int u = 0; u < IR_U; ++u)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                p0[u][j] = x[t0[u].o[j]];
                p1[u][j] = x[t1[u].o[j]];
            }
#pragma unroll
        for (int u = 0; u < IR_U; ++u) {
            const int b = b0 + u * NT;
            const real f0 = q0 * dv[u] * a_0[u] * t0[u].combine(p0[u][0], p0[u][1], p0[u][2], p0[u][3]);
            const real f1 = q1 * dv[u] * a_1[u] * t1[u].combine(p1[u][0], p1[u][1], p1[u][2], p1[u][3]);
            buf[b < nk ? (b - nk / 2) & (N - 1) : N] = cpx{f0, f1};
        }
    }
    twr.store(tws);
    __syncthreads();
    fft_lds<LOGN, 1, false>(buf, tws);
    cpx *R0 = R + (int64_t)item * g.r_stride + (int64_t)a0 * g.rw;
    cpx *R1 = R0 + g.rw;
    for (int kk = tid; kk <= N / 2; kk += NT) {
        const cpx z = buf[kk], zm = buf[(N - kk) & (N - 1)];
        // X = (Z + conj Zm)/2 (row a0), Y = (Z - conj Zm)/(2i) (row a0+1)
        R0[kk] = cpx{real(0.5) * (z.re + zm.re), real(0.5) * (z.im - zm.im)};
        R1[kk] = cpx{real(0.5) * (z.im + zm.im), real(0.5) * (zm.re - z.re)};
    }
}

// -------------------------------------------------------------- forward column pass
template <int LOGN, int CB>
__global__ __launch_bounds__(NT) void k_col_fwd(Geom g, const cpx *__restrict__ R,
                                                const cpx *__restrict__ tw, cpx *__restrict__ ext) {
    constexpr int N = 1 << LOGN;
    constexpr int MAXE = 8 * CB;
    __shared__ cpx buf[CB * N + 1]; // + a sink cell for the stores of positions past the end
    __shared__ cpx tws[tw_len<LOGN>()];
    TwStage<LOGN> twr;
    twr.fetch(tw);
    __shared__ int ent_col[MAXE];
    __shared__ int ent_src[MAXE];
    __shared__ int n_ent;
    const int tid = threadIdx.x;
    int item, c0;
    if (!col_block<CB>(g, item, c0)) return;
    const int nk = g.nk;
    for (int i = tid; i < CB * N; i += NT) buf[i] = cpx{0, 0};
    if (tid == 0) {
        // extended columns fed by this block's source columns: direct copies at
        // src + O + m N, Hermitian mirrors (conjugate, row-reversed) at N - src + O + m N
        int n = 0;
        for (int cc = 0; cc < CB; ++cc) {
            const int src = c0 + cc;
            if (src >= g.rw) break;
            for (int m = -2; m <= 2; ++m) {
                const int ec = src + g.O + m * N;
                if (ec >= 0 && ec < g.ew && n < MAXE) { ent_col[n] = ec; ent_src[n] = cc; ++n; }
            }
            if (src != 0 && src != N / 2) {
                for (int m = -2; m <= 2; ++m) {
                    const int ec = N - src + g.O + m * N;
                    if (ec >= 0 && ec < g.ew && n < MAXE) { ent_col[n] = ec; ent_src[n] = cc | 0x10000; ++n; }
                }
            }
        }
        n_ent = n;
    }
    __syncthreads();
    const cpx *Ri = R + (int64_t)item * g.r_stride;
    // COL_LOADS rows of the source per thread are requested before the first is stored, so
    // that a block keeps that many loads per lane in flight instead of one.  Loads and stores
    // are unconditional (positions past the end read element 0 and store to the sink cell):
    // with either behind a branch the compiler waits for each load before issuing the next.
    for (int e0 = tid; e0 < nk * CB; e0 += COL_LOADS * NT) {
        cpx v[COL_LOADS];
#pragma unroll
        for (int u = 0; u < COL_LOADS; ++u) {
            const int e = e0 + u * NT, a = e / CB, cc = e - (e / CB) * CB;
            const bool ok = e < nk * CB && c0 + cc < g.rw;
            v[u] = Ri[ok ? (int64_t)a * g.rw + c0 + cc : 0];
        }
#pragma unroll
        for (int u = 0; u < COL_LOADS; ++u) {
            const int e = e0 + u * NT, a = e / CB, cc = e - (e / CB) * CB;
            const bool ok = e < nk * CB && c0 + cc < g.rw;
            buf[ok ? ((a - nk / 2) & (N - 1)) * CB + cc : CB * N] = v[u];
        }
    }
    twr.store(tws);
    __syncthreads();
    fft_lds<LOGN, CB, false>(buf, tws);
    cpx *E = ext + (int64_t)item * g.ext_stride;
    const int ne = n_ent;
    for (int e = tid; e < ne * g.eh; e += NT) {
        const int en = e / g.eh, er = e - (e / g.eh) * g.eh;
        const int src = ent_src[en];
        const int cc = src & 0xFFFF;
        const int t1 = (er - g.O) & (N - 1);
        cpx v;
        if (src & 0x10000) {
            v = buf[((N - t1) & (N - 1)) * CB + cc];
            v.im = -v.im;
        } else {
            v = buf[t1 * CB + cc];
        }
        E[(int64_t)ent_col[en] * g.eh + er] = v; // column-major
    }
}

// ------------------------------------------------------------------- gridding kernel
// phi(z) = exp(beta (sqrt(1 - (2z/W)^2) - 1)).  In the float build the exponential is
// taken as exp2 of a prescaled argument (v_exp_f32, v_sqrt_f32): an argument error d
// changes phi by phi * d, and phi * |argument| never exceeds 1/e, so the absolute error
// stays at the rounding level of the peak weight.  beta2 = beta (double build) or
// beta * log2(e) (float build).
__device__ __forceinline__ real es_kernel(real z, real inv_half_w, real beta2) {
    const real t = z * inv_half_w;
    const real q = real(1) - t * t;
#ifdef IVX_REAL_DOUBLE
    return exp(beta2 * (sqrt(q > real(0) ? q : real(0)) - real(1)));
#else
    return __builtin_amdgcn_exp2f(beta2 * (__builtin_amdgcn_sqrtf(q > 0.f ? q : 0.f) - 1.f));
#endif
}

__device__ __forceinline__ void decode(const VisCoord &v, int &ix, int &iy, real &fx, real &fy) {
#ifdef IVX_REAL_DOUBLE
    ix = (int)v.ix;
    iy = (int)v.iy;
    fx = v.fx;
    fy = v.fy;
#else
    ix = (int)(v.xq >> 24);
    iy = (int)(v.yq >> 24);
    fx = (real)(v.xq & 0xFFFFFFu) * real(5.9604644775390625e-08); // 2^-24
    fy = (real)(v.yq & 0xFFFFFFu) * real(5.9604644775390625e-08);
#endif
}

struct GridArgs {
    Geom g;
    const WorkItem *work;
    const VisCoord *crd;
    const cpx *vis;
    const real *wgt;
    const int32_t *perm;
    const int64_t *boff;
    const cpx *ext;
    cpx *slots;
    double *jpart;
    const cpx *caller_in;
    cpx *caller_out;
    int nwave;
    int n_work;
    int unweighted; // adjoint mode: spread the given visibilities without the natural weights
    // w-plane modes
    const WZ *wz;
    cpx *wacc;
    const cpx *wq;
    int wplane;
    int wW;
    real wbeta2; // w kernel shape, scaled like beta2 below
    const int32_t *wcnt; // record counts below each half plane per work item, or NULL
    int wncnt;
    uint8_t *wsact;      // adjoint plane pass: slot written (1) or skipped (0), or NULL
};

// Signed distance, in planes, of a record's w from plane p.
__device__ __forceinline__ real wz_dist(WZ z, int p) {
#ifdef IVX_REAL_DOUBLE
    return z - (double)p;
#else
    return (real)((int)(z >> 24) - p) + (real)(z & 0xFFFFFFu) * real(5.9604644775390625e-08);
#endif
}

// First record of a work item's (sorted) list whose plane coordinate reaches the given
// number of half planes: lower bound of zeta >= h2 / 2.
__device__ __forceinline__ int wz_lower(const WZ *__restrict__ z, int n, int h2) {
#ifdef IVX_REAL_DOUBLE
    const double key = 0.5 * (double)h2;
#else
    const int64_t k = (int64_t)h2 << 23;
    if (k <= 0) return 0;
    if (k > (int64_t)0xFFFFFFFFll) return n;
    const uint32_t key = (uint32_t)k;
#endif
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (z[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Work items per row of the gridding launch: the dispatch packet counts work-items of one
// grid dimension in 32 bits, so long work lists (spectral cubes) wrap into blockIdx.y.
constexpr unsigned GRID_ROW = 1u << 22;

// ---- cross-lane moves inside a 16-lane DPP row (VALU, no LDS traffic)
// (mov_dpp with bound_ctrl: lanes without a source read 0, and no old value has to be
// materialised first)
template <int CTRL> __device__ __forceinline__ float dpp(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
template <int CTRL> __device__ __forceinline__ double dpp(double v) {
    const int2 p = __builtin_bit_cast(int2, v);
    int2 r;
    r.x = __builtin_amdgcn_mov_dpp(p.x, CTRL, 0xF, 0xF, true);
    r.y = __builtin_amdgcn_mov_dpp(p.y, CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, r);
}
template <int L> __device__ __forceinline__ real row_bcast(real v) { return dpp<0x150 + L>(v); }


__device__ __forceinline__ real row_shr8(real v) { return dpp<0x118>(v); }

// Lane layout of a G-lane group (one visibility at a time):
//   G = 8  (W <= 8): lane j owns footprint column j, all W rows (two groups per DPP row);
//   G = 16, W <= 8 : lane t owns column t & 7 and every other row starting at t >> 3;
//   G = 16, W > 8  : lane t < W owns column t, all W rows.
template <int W, int G> struct Layout {
    static_assert(G == 16 || W <= 8, "8-lane groups need W <= 8");
    static constexpr int S = (G == 16 && W <= 8) ? 2 : 1; // row stride of a lane
    static constexpr int NR = (W + S - 1) / S;            // rows per lane (upper bound)
};

// Row weights of the group in every lane: wsel[k] is the weight of the lane's k-th row.
template <int W, int G, int I> struct RowWeights {
    __device__ __forceinline__ static void run(real mine, bool upper, real *wsel) {
        if constexpr (G == 8) {
            const real lo = row_bcast<I>(mine), hi = row_bcast<8 + I>(mine);
            wsel[I] = upper ? hi : lo;
        } else if constexpr (Layout<W, G>::S == 2) {
            // rows 2k (lanes h = 0) and 2k + 1 (h = 1) come from lanes 8 + 2k and 8 + 2k + 1
            if constexpr (I % 2 == 0) {
                const real e0 = row_bcast<8 + I>(mine);
                const real e1 = (I + 1 < W) ? row_bcast<8 + ((I + 1 < W) ? I + 1 : I)>(mine) : real(0);
                wsel[I / 2] = upper ? e1 : e0;
            }
        } else {
            wsel[I] = row_bcast<I>(mine);
        }
        RowWeights<W, G, I + 1>::run(mine, upper, wsel);
    }
};
template <int W, int G> struct RowWeights<W, G, W> {
    __device__ __forceinline__ static void run(real, bool, real *) {}
};

// sum over the lanes of the group, returned in every lane of the group
template <int G> __device__ __forceinline__ real group_sum(real v) {
    v += dpp<0xB1>(v);  // quad xor 1
    v += dpp<0x4E>(v);  // quad xor 2
    v += dpp<0x141>(v); // half-row mirror: the other quad of the 8
    if constexpr (G == 16) v += dpp<0x140>(v); // row mirror: the other half
    return v;
}

// One block per work item (a fine-grid tile, or a chunk of one).  The block's waves split
// into groups of G lanes; group g walks its own contiguous segment of the tile's
// visibility list.  Inside a group the kernel weights are evaluated once (one or two per
// lane) and moved across lanes with DPP row operations, and the degridded value is a DPP
// group sum, so no cross-lane traffic touches the LDS.  Every group spreads into its own
// LDS accumulator window with plain read-modify-write (the lanes of a group own distinct
// cells and no other group writes there): no atomics.  The windows are summed in a fixed
// order at the end, so results do not depend on scheduling.
// LDS: F window (unless MODE_ADJ) + one accumulator window per group (unless MODE_FWD),
// each column-major with column stride ldw: the rows a lane owns in one footprint column
// are then a few cells apart, so their offsets are immediates of the LDS instructions.
template <int W, int MODE, int G, int VPI>
__global__ __launch_bounds__(NT) void k_grid(GridArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[NT / 64];
    constexpr int S = Layout<W, G>::S, NR = Layout<W, G>::NR;
    constexpr int GPW = 64 / G; // groups per wave
    const Geom &g = a.g;
    const int win = g.win, ldw = g.ldw;
    const int wsz = win * ldw;
    const int nwave = a.nwave;
    const int ngroups = nwave * GPW;
    cpx *Fw = reinterpret_cast<cpx *>(smem_raw);
    constexpr bool WPL = MODE == MODE_WFWD || MODE == MODE_WADJ; // one w plane of the full model
    constexpr bool NOGRID = MODE == MODE_ADJ || MODE == MODE_WADJ; // the grid window is not read
    constexpr bool SPREAD = MODE == MODE_OBJ || MODE == MODE_ADJ || MODE == MODE_WADJ;
    constexpr bool DATA = MODE == MODE_OBJ || MODE == MODE_VAL; // residual against the data
    cpx *Hw = Fw + (NOGRID ? 0 : wsz);
    const int64_t wid = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    if (wid >= a.n_work) return; // tail of the last row: the whole block leaves together
    const WorkItem wi = a.work[wid];
    const int tid = threadIdx.x;
    // e = cc * win + r without an integer division: (e + 1/2) / win is never within float
    // rounding of an integer for e < 2^16
    const float inv_win = 1.0f / (float)win;
    // a w plane only takes the records whose w kernel reaches it, zeta in [p - W_w / 2,
    // p + W_w / 2): a contiguous range of the work item's list (sorted by zeta).  Most work
    // items meet a plane with no such record: the degrid pass then has nothing to do and the
    // spread pass writes a zero window (the values are block-uniform, so the whole block
    // leaves together).
    int base = 0, cnt = wi.count;
    if constexpr (WPL) {
        const int h0 = 2 * a.wplane - a.wW, h1 = 2 * a.wplane + a.wW;
        if (a.wcnt) {
            // two independent loads from the work item's table instead of two chains of
            // dependent loads
            const int32_t *c = a.wcnt + wid * (int64_t)a.wncnt;
            base = h0 <= 0 ? 0 : (h0 >= a.wncnt ? wi.count : c[h0]);
            cnt = (h1 <= 0 ? 0 : (h1 >= a.wncnt ? wi.count : c[h1])) - base;
        } else {
            const WZ *z = a.wz + wi.begin;
            base = wz_lower(z, wi.count, h0);
            cnt = wz_lower(z, wi.count, h1) - base;
        }
        if (MODE == MODE_WADJ && a.wsact && tid == 0) a.wsact[wi.slot] = cnt > 0 ? 1 : 0;
        if (cnt == 0) {
            if (MODE == MODE_WADJ && !a.wsact) {
                cpx *Sl = a.slots + (int64_t)wi.slot * g.win_stride;
                for (int e = tid; e < win * win; e += blockDim.x) Sl[e] = cpx{0, 0};
            }
            return;
        }
    }
    if (!NOGRID) {
        const cpx *F = a.ext + (int64_t)wi.item * g.ext_stride + (int64_t)(wi.tx * g.T) * g.eh + wi.ty * g.T;
        for (int e = tid; e < win * win; e += blockDim.x) {
            const int cc = (int)(((float)e + 0.5f) * inv_win), r = e - cc * win;
            Fw[cc * ldw + r] = F[cc * g.eh + r];
        }
    }
    if (SPREAD) {
        for (int e = tid; e < ngroups * wsz; e += blockDim.x) Hw[e] = cpx{0, 0};
    }
    __syncthreads();

    const int lane = tid & 63, wave = tid >> 6;
    const int t = lane & (G - 1);
    const int j = (S == 2) ? (t & 7) : t;   // footprint column owned
    const int h = (S == 2) ? (t >> 3) : 0;  // first footprint row owned
    const bool upper = (lane & 8) != 0;      // second half of the DPP row
    const bool colok = j < W;
    const int gid = wave * GPW + lane / G;
    cpx *Hg = Hw + gid * wsz;
    const real inv_hw = real(2) / real(W);
#ifdef IVX_REAL_DOUBLE
    const real beta2 = g.beta;
#else
    const real beta2 = g.beta * 1.4426950408889634f;
#endif
    const real zoff = real(0.5) * real(W) - real(1);
    real jacc = real(0);

    // this group's segment of the tile's list (of the plane's range), walked VPI visibilities
    // at a time
    const int seg = (cnt + ngroups - 1) / ngroups;
    const int v0 = base + gid * seg;
    const int v1 = min(base + cnt, v0 + seg);
    const int nit = (seg + VPI - 1) / VPI;
    const VisCoord *crd = a.crd + wi.begin;
    const cpx *vis = a.vis + wi.begin;
    const real *wgt = a.wgt + wi.begin;
    const int32_t *perm = a.perm + wi.begin;
    cpx *caller_out = nullptr;
    const cpx *caller_in = nullptr;
    if (MODE == MODE_FWD) caller_out = a.caller_out + a.boff[wi.item];
    if (MODE == MODE_ADJ) caller_in = a.caller_in + a.boff[wi.item];
    // per-lane record index as an unsigned 32-bit byte offset from the block's (uniform)
    // bases, so the loads take the scalar-base + 32-bit vector-offset form
    auto rec = [&](int vv) -> unsigned { return (unsigned)(vv < v1 ? vv : 0); };
    auto at = [](const auto *base, unsigned i) {
        using T = std::remove_cv_t<std::remove_pointer_t<decltype(base)>>;
        return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + i * (unsigned)sizeof(T));
    };

    // record of one visibility (the fields this mode reads)
    struct Rec {
        VisCoord c;
        cpx y;
        real w;
        int32_t p;
    };
    auto load = [&](Rec (&r)[VPI], int it) {
#pragma unroll
        for (int u = 0; u < VPI; ++u) {
            const unsigned vn = rec(v0 + it * VPI + u);
            r[u].c = at(crd, vn);
            r[u].y = cpx{0, 0};
            r[u].w = real(0);
            r[u].p = 0;
            if (DATA) { r[u].y = at(vis, vn); r[u].w = at(wgt, vn); }
            if (MODE == MODE_ADJ) { r[u].w = a.unweighted ? real(1) : at(wgt, vn); r[u].p = at(perm, vn); }
            if (MODE == MODE_FWD) { r[u].p = at(perm, vn); }
            if constexpr (WPL) {
                // w carries the record's w-kernel weight for this plane, y its coefficient
                r[u].w = es_kernel(wz_dist(at(a.wz + wi.begin, vn), a.wplane), real(2) / real(a.wW), a.wbeta2);
                if (MODE == MODE_WADJ) r[u].y = at(a.wq + wi.begin, vn);
            }
        }
    };

    // one iteration: VPI visibilities of this group's segment
    auto step = [&](const Rec (&cur)[VPI], int it) {
        bool valid[VPI];
#pragma unroll
        for (int u = 0; u < VPI; ++u) valid[u] = v0 + it * VPI + u < v1;
        int off[VPI];
        real wxj[VPI], wsel[VPI][NR];
#pragma unroll
        for (int u = 0; u < VPI; ++u) {
            int ix, iy;
            real fx, fy;
            decode(cur[u].c, ix, iy, fx, fy);
            // kernel weights: x weight of the owned column, y weights of the owned rows
            if constexpr (G == 16 && S == 2) {
                // lanes 0-7 evaluate the column weights, lanes 8-15 the row weights; DPP row
                // moves hand every lane its column's weight and its rows' weights
                const bool isx = t < 8;
                const int k = t & 7;
                real mine = real(0);
                if (k < W) mine = es_kernel(zoff + (isx ? fx : fy) - real(k), inv_hw, beta2);
                const real sh = row_shr8(mine);
                wxj[u] = isx ? mine : sh;
                RowWeights<W, G, 0>::run(mine, upper, wsel[u]);
            } else if constexpr (G == 8) {
                real mx = real(0), my = real(0);
                if (colok) {
                    mx = es_kernel(zoff + fx - real(j), inv_hw, beta2);
                    my = es_kernel(zoff + fy - real(j), inv_hw, beta2);
                }
                wxj[u] = mx;
                RowWeights<W, G, 0>::run(my, upper, wsel[u]);
            } else {
                real mx = real(0), my = real(0);
                if (colok) {
                    mx = es_kernel(zoff + fx - real(j), inv_hw, beta2);
                    my = es_kernel(zoff + fy - real(j), inv_hw, beta2);
                }
                wxj[u] = mx;
                RowWeights<W, G, 0>::run(my, upper, wsel[u]);
            }
            if (!valid[u]) wxj[u] = real(0);
            off[u] = (int)__umul24((unsigned)(ix + j), (unsigned)ldw) + iy + h;
        }
        real ar[VPI], ai[VPI];
#pragma unroll
        for (int u = 0; u < VPI; ++u) {
            ar[u] = real(0);
            ai[u] = real(0);
        }
        if (!NOGRID) {
            if (colok) {
#pragma unroll
                for (int k = 0; k < NR; ++k) {
                    if (S == 1 || h + S * k < W) {
#pragma unroll
                        for (int u = 0; u < VPI; ++u) {
                            const cpx f = Fw[off[u] + S * k];
                            ar[u] += wsel[u][k] * f.re;
                            ai[u] += wsel[u][k] * f.im;
                        }
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < VPI; ++u) {
                ar[u] = group_sum<G>(ar[u] * wxj[u]);
                ai[u] = group_sum<G>(ai[u] * wxj[u]);
            }
        }
        if (MODE == MODE_FWD) {
#pragma unroll
            for (int u = 0; u < VPI; ++u) {
                if (valid[u] && t == 0) {
                    if (cur[u].p < 0) caller_out[~cur[u].p] = cpx{ar[u], -ai[u]};
                    else caller_out[cur[u].p] = cpx{ar[u], ai[u]};
                }
            }
            return;
        }
        if (MODE == MODE_WFWD) {
            // planes run as successive launches and a record belongs to one group of one work
            // item: a plain read-modify-write, in plane order
#pragma unroll
            for (int u = 0; u < VPI; ++u) {
                if (valid[u] && t == 0) {
                    cpx *o = a.wacc + wi.begin + (v0 + it * VPI + u);
                    cpx ov = *o;
                    ov.re += cur[u].w * ar[u];
                    ov.im += cur[u].w * ai[u];
                    *o = ov;
                }
            }
            return;
        }
        real cre[VPI], cim[VPI];
#pragma unroll
        for (int u = 0; u < VPI; ++u) {
            if (DATA) {
                const real rr = ar[u] - cur[u].y.re, ri = ai[u] - cur[u].y.im;
                if (valid[u] && t == 0) jacc += cur[u].w * (rr * rr + ri * ri); // halved at the end
                const real ww = cur[u].w * wxj[u];
                cre[u] = ww * rr;
                cim[u] = ww * ri;
            } else if (MODE == MODE_WADJ) {
                cre[u] = cur[u].w * cur[u].y.re * wxj[u];
                cim[u] = cur[u].w * cur[u].y.im * wxj[u];
            } else {
                cpx y = caller_in[cur[u].p < 0 ? ~cur[u].p : cur[u].p];
                if (cur[u].p < 0) y.im = -y.im;
                cre[u] = cur[u].w * y.re * wxj[u];
                cim[u] = cur[u].w * y.im * wxj[u];
            }
        }
        // spread: the visibilities of one iteration go in program order, so a cell shared
        // by two of them (owned by different lanes) sees both updates
        if (SPREAD && colok) {
#pragma unroll
            for (int u = 0; u < VPI; ++u) {
#pragma unroll
                for (int k = 0; k < NR; ++k) {
                    if (S == 1 || h + S * k < W) {
                        cpx *hp = Hg + off[u] + S * k;
                        cpx hv = *hp;
                        hv.re += cre[u] * wsel[u][k];
                        hv.im += cim[u] * wsel[u][k];
                        *hp = hv;
                    }
                }
            }
        }
    };

    // three record sets rotate: the records of iteration it + 2 are requested as iteration
    // it starts, two iterations of latency cover (no register copies between stages)
    Rec r0[VPI], r1[VPI], r2[VPI];
    load(r0, 0);
    load(r1, 1);
    for (int it = 0; it < nit; it += 3) {
        if (it + 2 < nit) load(r2, it + 2);
        step(r0, it);
        if (it + 1 >= nit) break;
        if (it + 3 < nit) load(r0, it + 3);
        step(r1, it + 1);
        if (it + 2 >= nit) break;
        if (it + 4 < nit) load(r1, it + 4);
        step(r2, it + 2);
    }
    if (MODE == MODE_FWD || MODE == MODE_WFWD) return;
    if (SPREAD) {
        __syncthreads();
        cpx *Sl = a.slots + (int64_t)wi.slot * g.win_stride; // column-major window
        for (int e = tid; e < win * win; e += blockDim.x) {
            const int cc = (int)(((float)e + 0.5f) * inv_win), r = e - cc * win;
            real sr = real(0), si = real(0);
            for (int q = 0; q < ngroups; ++q) {
                const cpx hh = Hw[q * wsz + cc * ldw + r];
                sr += hh.re;
                si += hh.im;
            }
            Sl[e] = cpx{sr, si};
        }
    }
    if (DATA) {
        double d = 0.5 * (double)jacc;
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) d += __shfl_xor(d, m, 64);
        if (lane == 0) red[wave] = d;
        __syncthreads();
        if (tid == 0) {
            double sacc = 0.0;
            for (int w = 0; w < nwave; ++w) sacc += red[w];
            a.jpart[wid] = sacc;
        }
    }
}

int grid_groups_per_wave(int W, int lanes) { return (lanes == 8 && W <= 8) ? 8 : 4; }

#ifndef IVX_REAL_DOUBLE
// ---------------------------------------------------- gridding on the matrix cores
// The same degrid / residual / spread as k_grid, written as per-tile matrix products (float
// build, windows of at most 16 x 16 cells).  One wave per work item; per batch of 16
// visibilities the kernel weights of every visibility at the 16 window columns (PX[m][b])
// and rows (PY[m][a]) -- zero outside its footprint -- go to LDS, then
//   degrid   Q[a][m] = sum_b F[a][b] PX[m][b]              (v_mfma_f32_16x16x4_f32, K = b)
//            V_m     = sum_a PY[m][a] Q[a][m]              (4 rows per lane + two lane swaps)
//   spread   H[a][b] += sum_m PY[m][a] (w_m r_m) PX[m][b]  (v_mfma_f32_16x16x4_f32, K = m)
// The window F and the accumulation H stay in registers for the whole work item; H is
// written to the work item's slot at the end.  Operand layout of the 16x16x4 instruction:
// lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and receives D[4 (l / 16) + v][l % 16].
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int MX_LD = 17; // row stride of the weight tables (bank spread)

// LDS hand-off between the lanes of the (single-wave) block: a wave's LDS operations are
// performed in order, so only the compiler has to be kept from moving accesses across;
// unlike a block barrier this does not wait for the wave's outstanding global loads.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sum of x over the four 16-lane rows, returned in every lane of the column (lanes l, l ^ 16,
// l ^ 32, l ^ 48), with the VALU row swaps of gfx950 instead of LDS permutes.  Swapping the
// odd rows of one copy with the even rows of another and adding gives x[r] + x[r ^ 1] in row
// r; the same with row pairs {2, 3} <-> {0, 1} completes the sum.  The additions pair the
// same operands as two xor-shuffle steps (16, then 32), so the result is bitwise the same.
__device__ __forceinline__ float row_sum4(float x) {
    const unsigned u = __float_as_uint(x);
    const auto p = __builtin_amdgcn_permlane16_swap(u, u, false, false);
    const float y = __uint_as_float(p[0]) + __uint_as_float(p[1]);
    const unsigned v = __float_as_uint(y);
    const auto q = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return __uint_as_float(q[0]) + __uint_as_float(q[1]);
}

// KW > 0 fixes the kernel width at compile time (the footprint loops unroll without
// per-lane width tests); KW = 0 reads it from the geometry.  OCC is the occupancy the
// register allocation aims for: 7 waves per SIMD (72 VGPRs) pays on launches of many work
// items, 6 (a freer schedule) on launches that fill the chip about once.
// The w-plane modes of the full model take, as the vector gridder's do, the plane's range of
// the work item's records (sorted by plane coordinate) and weigh each record by its w kernel
// at the plane: MODE_WFWD adds w_p V_m to the record's accumulator, MODE_WADJ spreads
// w_p q_m (q the record's adjoint coefficient).
template <int MODE, int KW, int OCC>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(OCC, 8))) void k_gridmx(GridArgs a) {
    __shared__ float PX[16 * MX_LD], PY[16 * MX_LD];
    __shared__ float WRr[16], WRi[16];
    const int64_t wid = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    if (wid >= a.n_work) return;
    const WorkItem wi = a.work[wid];
    if (wi.count <= 0) return; // (the work list holds no empty items)
    const Geom &g = a.g;
    const int l = threadIdx.x, c16 = l & 15, g4 = l >> 4;
    const int W = KW > 0 ? KW : g.W, win = g.win;
    constexpr bool WPL = MODE == MODE_WFWD || MODE == MODE_WADJ; // one w plane of the full model
    constexpr bool NOGRID = MODE == MODE_ADJ || MODE == MODE_WADJ; // the grid window is not read
    constexpr bool SPREAD = MODE == MODE_OBJ || MODE == MODE_ADJ || MODE == MODE_WADJ;
    constexpr bool DATA = MODE == MODE_OBJ || MODE == MODE_VAL; // residual against the data
    // the records of this work item that the pass takes: all, or the plane's range
    int base = 0, n = wi.count;
    if constexpr (WPL) {
        const int h0 = 2 * a.wplane - a.wW, h1 = 2 * a.wplane + a.wW;
        if (a.wcnt) {
            const int32_t *c = a.wcnt + wid * (int64_t)a.wncnt;
            base = h0 <= 0 ? 0 : (h0 >= a.wncnt ? wi.count : c[h0]);
            n = (h1 <= 0 ? 0 : (h1 >= a.wncnt ? wi.count : c[h1])) - base;
        } else {
            const WZ *z = a.wz + wi.begin;
            base = wz_lower(z, wi.count, h0);
            n = wz_lower(z, wi.count, h1) - base;
        }
        if (MODE == MODE_WADJ && a.wsact && l == 0) a.wsact[wi.slot] = n > 0 ? 1 : 0;
        if (n == 0) { // (uniform over the wave) no record near the plane: no window, or a zero one
            if (MODE == MODE_WADJ && !a.wsact) {
                cpx *Sl = a.slots + (int64_t)wi.slot * g.win_stride;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = 4 * g4 + v;
                    if (r < win && c16 < win) Sl[c16 * win + r] = cpx{0.f, 0.f};
                }
            }
            return;
        }
    }
    const float zoff = 0.5f * (float)W - 1.f;
    const float inv_hw = 2.f / (float)W;
    const float beta2 = g.beta * 1.4426950408889634f;
    // window F[a][b] (tile rows a, columns b), lane holds F[c16][4 i + g4]
    float fr[4] = {0.f, 0.f, 0.f, 0.f}, fi[4] = {0.f, 0.f, 0.f, 0.f};
    if (!NOGRID) {
        const cpx *F = a.ext + (int64_t)wi.item * g.ext_stride + (int64_t)(wi.tx * g.T) * g.eh + wi.ty * g.T;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int b = 4 * i + g4;
            if (c16 < win && b < win) {
                const cpx v = F[b * g.eh + c16];
                fr[i] = v.re;
                fi[i] = v.im;
            }
        }
    }
    f32x4 hre = {0.f, 0.f, 0.f, 0.f}, him = {0.f, 0.f, 0.f, 0.f};
    float jacc = 0.f;
    const VisCoord *crd = a.crd + wi.begin + base;
    const cpx *vis = a.vis + wi.begin;
    const real *wgt = a.wgt + wi.begin;
    const int32_t *perm = a.perm + wi.begin;
    const WZ *wzp = WPL ? a.wz + wi.begin + base : nullptr;
    cpx *wacc = MODE == MODE_WFWD ? a.wacc + wi.begin + base : nullptr;
    const cpx *wq = MODE == MODE_WADJ ? a.wq + wi.begin + base : nullptr;
    const float inv_hww = WPL ? 2.f / (float)a.wW : 0.f;
    cpx *caller_out = nullptr;
    const cpx *caller_in = nullptr;
    if (MODE == MODE_FWD) caller_out = a.caller_out + a.boff[wi.item];
    if (MODE == MODE_ADJ) caller_in = a.caller_in + a.boff[wi.item];
    // records of a batch (lanes 0-15); two sets rotate so that the next batch's records are
    // in flight while the current batch is processed, with no register copies
    struct MxRec {
        VisCoord c; // coordinates of visibility l / 4 of the batch (every lane)
        cpx y;      // data, weight, caller index of visibility l (lanes 0-15)
        float w;
        int p;
    };
    // Every lane loads, at indices clamped to the last record (a batch past the end reloads
    // it and ignores it): with no per-lane branches around the loads the wait before a batch
    // covers only that batch's own loads, not the prefetch issued just before it.
    auto fetch = [&](MxRec &r, int v0) {
        const int vi = min(v0 + c16, n - 1), vw = min(v0 + (l >> 2), n - 1);
        r.c = crd[vw];
        if (DATA) { r.y = vis[vi]; r.w = wgt[vi]; }
        if (MODE == MODE_ADJ) { r.w = a.unweighted ? 1.f : wgt[vi]; r.p = perm[vi]; }
        if (MODE == MODE_FWD) r.p = perm[vi];
        if constexpr (WPL) {
            // w carries the record's w-kernel weight at this plane, y its coefficient
            r.w = es_kernel(wz_dist(wzp[vi], a.wplane), inv_hww, a.wbeta2);
            if (MODE == MODE_WADJ) r.y = wq[vi];
        }
    };
    auto batch = [&](const MxRec &r, int v0) {
        const bool ok = l < 16 && v0 + c16 < n;
        if (MODE == MODE_ADJ && l < 16) {
            float yr = 0.f, yi = 0.f;
            if (ok) {
                const cpx y = caller_in[r.p < 0 ? ~r.p : r.p];
                yr = r.w * y.re;
                yi = r.w * (r.p < 0 ? -y.im : y.im);
            }
            WRr[l] = yr;
            WRi[l] = yi;
        }
        if (MODE == MODE_WADJ && l < 16) {
            WRr[l] = ok ? r.w * r.y.re : 0.f;
            WRi[l] = ok ? r.w * r.y.im : 0.f;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int e = l + 64 * i, m = e >> 4, pos = e & 15;
            PX[m * MX_LD + pos] = 0.f;
            PY[m * MX_LD + pos] = 0.f;
        }
        wave_sync();
        {
            // the W nonzero weights per visibility and axis: lane (m = l / 4, k = l % 4 + 4 j),
            // from the coordinates each lane decoded itself (no hand-off through LDS)
            const int m = l >> 2;
            if (v0 + m < n) {
                int ixm, iym;
                real fx, fy;
                decode(r.c, ixm, iym, fx, fy);
                const float zxm = zoff + fx, zym = zoff + fy;
#pragma unroll
                for (int j = 0; j < (KW > 0 ? (KW + 3) / 4 : 4); ++j) {
                    const int k = (l & 3) + 4 * j;
                    if ((KW > 0 && 4 * j + 3 < KW) || k < W) {
                        PX[m * MX_LD + ixm + k] = es_kernel(zxm - (float)k, inv_hw, beta2);
                        PY[m * MX_LD + iym + k] = es_kernel(zym - (float)k, inv_hw, beta2);
                    }
                }
            }
        }
        wave_sync();
        if (!NOGRID) {
            f32x4 qre = {0.f, 0.f, 0.f, 0.f}, qim = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float bx = PX[c16 * MX_LD + 4 * i + g4];
                qre = __builtin_amdgcn_mfma_f32_16x16x4f32(fr[i], bx, qre, 0, 0, 0);
                qim = __builtin_amdgcn_mfma_f32_16x16x4f32(fi[i], bx, qim, 0, 0, 0);
            }
            float vr = 0.f, vi = 0.f;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float py = PY[c16 * MX_LD + 4 * g4 + v];
                vr += py * qre[v];
                vi += py * qim[v];
            }
            vr = row_sum4(vr);
            vi = row_sum4(vi);
            // every lane now holds V of visibility c16 of the batch
            if (MODE == MODE_FWD) {
                if (ok) caller_out[r.p < 0 ? ~r.p : r.p] = cpx{vr, r.p < 0 ? -vi : vi};
                wave_sync();
                return;
            }
            if (MODE == MODE_WFWD) {
                // planes run as successive launches and a record belongs to one work item: a
                // plain read-modify-write, in plane order
                if (l < 16 && ok) {
                    cpx ov = wacc[v0 + c16];
                    ov.re += r.w * vr;
                    ov.im += r.w * vi;
                    wacc[v0 + c16] = ov;
                }
                wave_sync();
                return;
            }
            if (l < 16) {
                const float rr = vr - r.y.re, ri = vi - r.y.im;
                if (ok) jacc += r.w * (rr * rr + ri * ri); // halved at the end
                if (SPREAD) {
                    WRr[l] = ok ? r.w * rr : 0.f;
                    WRi[l] = ok ? r.w * ri : 0.f;
                }
            }
            wave_sync();
            if (!SPREAD) return;
        }
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            const int m = 4 * s4 + g4;
            const float ay = PY[m * MX_LD + c16];
            const float bx = PX[m * MX_LD + c16];
            hre = __builtin_amdgcn_mfma_f32_16x16x4f32(ay, WRr[m] * bx, hre, 0, 0, 0);
            him = __builtin_amdgcn_mfma_f32_16x16x4f32(ay, WRi[m] * bx, him, 0, 0, 0);
        }
        wave_sync(); // the tables are rewritten by the next batch
    };
    MxRec ra{}, rb{};
    fetch(ra, 0);
    for (int v0 = 0; v0 < n; v0 += 32) {
        fetch(rb, v0 + 16);
        batch(ra, v0);
        if (v0 + 16 >= n) break;
        fetch(ra, v0 + 32);
        batch(rb, v0 + 16);
    }
    if (MODE == MODE_FWD || MODE == MODE_WFWD) return;
    if (SPREAD) {
        cpx *Sl = a.slots + (int64_t)wi.slot * g.win_stride; // column-major window
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = 4 * g4 + v;
            if (r < win && c16 < win) Sl[c16 * win + r] = cpx{hre[v], him[v]};
        }
    }
    if (DATA) {
        double d = 0.5 * (double)jacc;
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) d += __shfl_xor(d, m, 64);
        if (l == 0) a.jpart[wid] = d;
    }
}
#endif

// ----------------------------------------------------------------------- fold
// Two passes.  (1) k_ext_sum: the adjoint extended grid E = sum of every work item's
// window placed at its tile, computed owner-wise: the block of (virtual) tile (vy, vx)
// owns the T x T cells starting at (vy T, vx T), which only the windows of tiles
// (vy - dy, vx - dx), dy, dx in {0, 1}, reach (a window spans T + W - 1 <= 2T cells);
// their slot lists are uniform per block and the window reads are contiguous along
// rows.  E overwrites the forward extended grid, which the gridding pass has consumed.
// (2) in the adjoint column pass, every half-plane cell sums the extended-grid cells that
// alias to it (periodic rows and columns) and is symmetrised, Hs = (H(t) + conj H(-t)) / 2,
// as it is loaded for the inverse column FFT.
constexpr int FOLD_LOADS = 8; // slot loads per thread in flight in k_ext_sum

__global__ __launch_bounds__(NT) void k_ext_sum(Geom g, int tiles_per_block, const int32_t *__restrict__ tslot,
                                                const cpx *__restrict__ slots, const uint8_t *__restrict__ sact,
                                                cpx *__restrict__ E) {
    const int item = blockIdx.y;
    const int T = g.T, win = g.win, TT = T * T;
    const int nvx = g.ntx + 1, nvt = (g.nty + 1) * nvx;
    // several small virtual tiles per block so that every thread owns a cell
    const int sub = threadIdx.x / TT;
    const int vt = blockIdx.x * tiles_per_block + sub;
    if (sub >= tiles_per_block || vt >= nvt) return;
    const int vy = vt / nvx, vx = vt - (vt / nvx) * nvx;
    const int32_t *ts = tslot + (int64_t)item * (g.nty * g.ntx + 1);
    int s_lo[4], s_hi[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int ty = vy - (q >> 1), tx = vx - (q & 1);
        s_lo[q] = s_hi[q] = 0;
        if (ty >= 0 && tx >= 0 && ty < g.nty && tx < g.ntx) {
            s_lo[q] = ts[ty * g.ntx + tx];
            s_hi[q] = ts[ty * g.ntx + tx + 1];
        }
    }
    const float inv_t = 1.0f / (float)T;
    cpx *Ei = E + (int64_t)item * g.ext_stride;
    for (int e = threadIdx.x - sub * TT; e < TT; e += NT) {
        const int c = (int)(((float)e + 0.5f) * inv_t), r = e - c * T;
        const int er = vy * T + r, ec = vx * T + c;
        if (er >= g.eh || ec >= g.ew) continue;
        // the (quadrant, slot) terms of the cell in one list, quadrant-major: FOLD_LOADS of
        // them are loaded at a time and then added in list order (the order of a plain
        // quadrant-by-quadrant, slot-by-slot sum)
        int off[4], p[5];
        p[0] = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int lr = r + (q >> 1) * T, lc = c + (q & 1) * T;
            const bool in = lr < win && lc < win;
            off[q] = lc * win + lr;
            p[q + 1] = p[q] + (in ? s_hi[q] - s_lo[q] : 0);
        }
        real sr = real(0), si = real(0);
        for (int i0 = 0; i0 < p[4]; i0 += FOLD_LOADS) {
            cpx h[FOLD_LOADS];
            int sl[FOLD_LOADS], oo[FOLD_LOADS];
            bool on[FOLD_LOADS];
#pragma unroll
            for (int u = 0; u < FOLD_LOADS; ++u) {
                const int i = i0 + u;
                const int q = (i >= p[1]) + (i >= p[2]) + (i >= p[3]);
                const int pq = q == 0 ? p[0] : q == 1 ? p[1] : q == 2 ? p[2] : p[3];
                const int lo = q == 0 ? s_lo[0] : q == 1 ? s_lo[1] : q == 2 ? s_lo[2] : s_lo[3];
                oo[u] = q == 0 ? off[0] : q == 1 ? off[1] : q == 2 ? off[2] : off[3];
                sl[u] = lo + i - pq;
                on[u] = i < p[4];
            }
            // the flags and the windows of the batch are requested together (one memory latency
            // per batch, not two); a window that was not written this pass may hold anything and
            // is dropped by the select, never added
            uint8_t f[FOLD_LOADS];
#pragma unroll
            for (int u = 0; u < FOLD_LOADS; ++u) {
                f[u] = 1;
                if (on[u]) {
                    if (sact) f[u] = sact[sl[u]];
                    h[u] = slots[(int64_t)sl[u] * g.win_stride + oo[u]];
                }
            }
#pragma unroll
            for (int u = 0; u < FOLD_LOADS; ++u) {
                if (on[u] && f[u]) {
                    sr += h[u].re;
                    si += h[u].im;
                }
            }
        }
        Ei[(int64_t)ec * g.eh + er] = cpx{sr, si};
    }
}

__device__ __forceinline__ cpx alias_sum(const Geom &g, const cpx *__restrict__ Ei, int t1, int t2) {
    const int msk = g.nf - 1;
    real sr = real(0), si = real(0);
    for (int ec = (t2 + g.O) & msk; ec < g.ew; ec += g.nf)
        for (int er = (t1 + g.O) & msk; er < g.eh; er += g.nf) {
            const cpx h = Ei[(int64_t)ec * g.eh + er];
            sr += h.re;
            si += h.im;
        }
    return cpx{sr, si};
}

// alias_sum for grids whose extended rows stop below 2 n_f and columns below n_f: the cell's
// column exists at most once and its row at most twice.  alias_pair loads the (up to) two
// values; pair_sum adds them in alias_sum's order (starting from zero, so a lone -0 reads
// as +0 there as well).
__device__ __forceinline__ void alias_pair(const Geom &g, const cpx *__restrict__ Ei, int t1, int t2, cpx &a,
                                           cpx &b) {
    const int msk = g.nf - 1;
    const int ec = (t2 + g.O) & msk, er = (t1 + g.O) & msk;
    if (ec < g.ew) {
        const cpx *col = Ei + (int64_t)ec * g.eh;
        if (er < g.eh) a = col[er];
        if (er + g.nf < g.eh) b = col[er + g.nf];
    }
}

__device__ __forceinline__ cpx pair_sum(const Geom &g, int t1, int t2, cpx a, cpx b) {
    const int msk = g.nf - 1;
    const int ec = (t2 + g.O) & msk, er = (t1 + g.O) & msk;
    real sr = real(0), si = real(0);
    if (ec < g.ew) {
        if (er < g.eh) { sr += a.re; si += a.im; }
        if (er + g.nf < g.eh) { sr += b.re; si += b.im; }
    }
    return cpx{sr, si};
}

// ------------------------------------------------------------ adjoint column pass
template <int LOGN, int CB>
__global__ __launch_bounds__(NT) void k_col_inv(Geom g, const cpx *__restrict__ E,
                                                const cpx *__restrict__ tw, cpx *__restrict__ R) {
    constexpr int N = 1 << LOGN;
    __shared__ cpx buf[CB * N];
    __shared__ cpx tws[tw_len<LOGN>()];
    TwStage<LOGN> twr;
    twr.fetch(tw);
    const int tid = threadIdx.x;
    int item, c0;
    if (!col_block<CB>(g, item, c0)) return;
    const cpx *Ei = E + (int64_t)item * g.ext_stride;
    if (g.eh <= 2 * g.nf && g.ew <= g.nf) {
        // every cell has at most two aliases (rows t and t + n_f of one column): the loads of
        // COL_LOADS cells are issued together, then summed in the order of alias_sum
        for (int e0 = tid; e0 < N * CB; e0 += COL_LOADS * NT) {
            cpx h0[COL_LOADS], h1[COL_LOADS], m0[COL_LOADS], m1[COL_LOADS];
#pragma unroll
            for (int u = 0; u < COL_LOADS; ++u) {
                const int e = e0 + u * NT, cc = e >> LOGN, t1 = e & (N - 1), t2 = c0 + cc;
                h0[u] = h1[u] = m0[u] = m1[u] = cpx{0, 0};
                if (e < N * CB && t2 < g.rw) {
                    alias_pair(g, Ei, t1, t2, h0[u], h1[u]);
                    alias_pair(g, Ei, (N - t1) & (N - 1), (N - t2) & (N - 1), m0[u], m1[u]);
                }
            }
#pragma unroll
            for (int u = 0; u < COL_LOADS; ++u) {
                const int e = e0 + u * NT, cc = e >> LOGN, t1 = e & (N - 1), t2 = c0 + cc;
                if (e >= N * CB) break;
                cpx v = cpx{0, 0};
                if (t2 < g.rw) {
                    const cpx h = pair_sum(g, t1, t2, h0[u], h1[u]);
                    const cpx m = pair_sum(g, (N - t1) & (N - 1), (N - t2) & (N - 1), m0[u], m1[u]);
                    v = cpx{real(0.5) * (h.re + m.re), real(0.5) * (h.im - m.im)};
                }
                buf[t1 * CB + cc] = v;
            }
        }
    } else {
        for (int e = tid; e < N * CB; e += NT) {
            const int cc = e >> LOGN, t1 = e & (N - 1);
            const int t2 = c0 + cc;
            cpx v = cpx{0, 0};
            if (t2 < g.rw) {
                const cpx h = alias_sum(g, Ei, t1, t2);
                const cpx m = alias_sum(g, Ei, (N - t1) & (N - 1), (N - t2) & (N - 1));
                v = cpx{real(0.5) * (h.re + m.re), real(0.5) * (h.im - m.im)};
            }
            buf[t1 * CB + cc] = v;
        }
    }
    twr.store(tws);
    __syncthreads();
    fft_lds<LOGN, CB, true>(buf, tws);
    cpx *Ri = R + (int64_t)item * g.r_stride;
    const int nk = g.nk;
    for (int e = tid; e < nk * CB; e += NT) {
        const int a = e / CB, cc = e - (e / CB) * CB;
        if (c0 + cc < g.rw) Ri[(int64_t)a * g.rw + c0 + cc] = buf[((a - nk / 2) & (N - 1)) * CB + cc];
    }
}

// ------------------------------------------- adjoint column pass straight from the slots
// k_ext_sum followed by k_col_inv without the extended grid in between: the block of a column
// group forms every extended cell its columns need from the slots that cover it (quadrant by
// quadrant, slot by slot, as k_ext_sum adds them), adds the second row alias and the
// Hermitian mirror in the order of k_col_inv, and runs the inverse column FFT.  The slot
// columns of a cell's tile are read by the one block that owns the cell's column, as whole
// 8-byte-per-row runs, instead of being written to and read back from the extended grid.
// Valid when every cell has at most two row aliases and one column alias (eh <= 2 n_f,
// ew <= n_f); the launcher falls back to the two-kernel path otherwise.

// Slot range and in-window offset of quadrant q of extended cell (er, ec): the window of tile
// (er / T - (q >> 1), ec / T - (q & 1)) covers the cell when the offset stays in the window.
__device__ __forceinline__ void cell_quadrant(const Geom &g, const int32_t *__restrict__ ts, int er, int ec, int q,
                                              int &lo, int &cnt, int &off) {
    const int vy = er / g.T, vx = ec / g.T;
    const int r = er - vy * g.T, c = ec - vx * g.T;
    const int ty = vy - (q >> 1), tx = vx - (q & 1);
    const int lr = r + (q >> 1) * g.T, lc = c + (q & 1) * g.T;
    lo = 0;
    cnt = 0;
    off = lc * g.win + lr;
    if (ty >= 0 && tx >= 0 && ty < g.nty && tx < g.ntx && lr < g.win && lc < g.win) {
        lo = ts[ty * g.ntx + tx];
        cnt = ts[ty * g.ntx + tx + 1] - lo;
    }
}

// Extended cell (er, ec) summed from the slots, in k_ext_sum's order (cells outside the
// extended grid are 0).
__device__ __forceinline__ cpx ext_cell(const Geom &g, const int32_t *__restrict__ ts, const cpx *__restrict__ slots,
                                        int er, int ec) {
    real sr = real(0), si = real(0);
    if (er >= g.eh || ec >= g.ew) return cpx{sr, si};
    for (int q = 0; q < 4; ++q) {
        int lo, cnt, off;
        cell_quadrant(g, ts, er, ec, q, lo, cnt, off);
        for (int k = 0; k < cnt; ++k) {
            const cpx h = slots[(int64_t)(lo + k) * g.win_stride + off];
            sr += h.re;
            si += h.im;
        }
    }
    return cpx{sr, si};
}

// alias_pair + pair_sum of k_col_inv with the cells formed from the slots.
__device__ __forceinline__ cpx alias_from_slots(const Geom &g, const int32_t *__restrict__ ts,
                                                const cpx *__restrict__ slots, int t1, int t2) {
    const int msk = g.nf - 1;
    const int ec = (t2 + g.O) & msk, er = (t1 + g.O) & msk;
    real sr = real(0), si = real(0);
    if (ec < g.ew) {
        if (er < g.eh) {
            const cpx a = ext_cell(g, ts, slots, er, ec);
            sr += a.re;
            si += a.im;
        }
        if (er + g.nf < g.eh) {
            const cpx b = ext_cell(g, ts, slots, er + g.nf, ec);
            sr += b.re;
            si += b.im;
        }
    }
    return cpx{sr, si};
}

// Cells per thread whose slot loads are in flight together, and columns per block of the fused
// pass: two and two measured fastest on the spectral cube (four cells per thread, or wider
// blocks, cost registers or LDS and with them the loads in flight per compute unit).
#ifndef IVX_FOLD_CELLS
#define IVX_FOLD_CELLS 2
#endif
#ifndef IVX_FOLD_CB
#define IVX_FOLD_CB 2
#endif
constexpr int FOLD_CELLS = IVX_FOLD_CELLS;

template <int LOGN, int CB>
__global__ __launch_bounds__(NT) void k_col_inv_slots(Geom g, const int32_t *__restrict__ tslot,
                                                      const cpx *__restrict__ slots, const cpx *__restrict__ tw,
                                                      cpx *__restrict__ R) {
    constexpr int N = 1 << LOGN;
    // tile rows of the grid: (n_f + O) / T + 1 with T >= 4 and O <= 8
    constexpr int MAXROWS = (N + 8) / 4 + 2;
    __shared__ cpx buf[CB * N];
    __shared__ cpx tws[tw_len<LOGN>()];
    // slot-list prefix of tile columns vxa - 1 .. vxa + 2 in every tile row: the tiles whose
    // windows reach this block's columns (CB <= T consecutive columns lie in at most two
    // tile columns)
    __shared__ int rng[MAXROWS + 1][4]; // + a sink row for the stores of entries past the end
    TwStage<LOGN> twr;
    twr.fetch(tw);
    const int tid = threadIdx.x;
    int item, c0;
    if (!col_block<CB>(g, item, c0)) return;
    const int32_t *ts = tslot + (int64_t)item * (g.nty * g.ntx + 1);
    const int msk = N - 1;
    const int vxa = (c0 + g.O) / g.T;
    // the prefix entries, RNG_U per thread requested together (loads clamped to entry 0,
    // stores past the end into the sink row; a guarded load would wait for the previous one)
    constexpr int RNG_U = 2;
    for (int e0 = tid; e0 < g.nty * 4; e0 += RNG_U * NT) {
        int32_t pv[RNG_U];
#pragma unroll
        for (int u = 0; u < RNG_U; ++u) {
            const int e = e0 + u * NT, ty = e >> 2, tx = vxa - 1 + (e & 3);
            const bool ok = e < g.nty * 4 && tx >= 0 && tx <= g.ntx;
            pv[u] = ts[ok ? ty * g.ntx + tx : 0];
        }
#pragma unroll
        for (int u = 0; u < RNG_U; ++u) {
            const int e = e0 + u * NT, ty = e >> 2, tx = vxa - 1 + (e & 3);
            const bool ok = e < g.nty * 4 && tx >= 0 && tx <= g.ntx;
            rng[e < g.nty * 4 ? ty : MAXROWS][e & 3] = ok ? pv[u] : 0;
        }
    }
    // the item's first slot (a valid address for the loads of empty quadrants), if it has any
    const int32_t s_first = ts[0];
    const bool any_slot = ts[g.nty * g.ntx] > s_first;
    __syncthreads();
    const float inv_t = 1.0f / (float)g.T;
    for (int e0 = tid; e0 < N * CB; e0 += FOLD_CELLS * NT) {
        // the quadrant lists of FOLD_CELLS cells (first row alias) from the LDS table, then
        // the first slot of every quadrant of every cell requested together, then the sums in
        // k_ext_sum's order
        int lo[FOLD_CELLS][4], cnt[FOLD_CELLS][4], off[FOLD_CELLS][4];
        cpx first[FOLD_CELLS][4];
#pragma unroll
        for (int u = 0; u < FOLD_CELLS; ++u) {
            const int e = e0 + u * NT, cc = e >> LOGN, t1 = e & msk, t2 = c0 + cc;
            const int er = (t1 + g.O) & msk, ec = (t2 + g.O) & msk;
            const bool live = e < N * CB && t2 < g.rw && er < g.eh && ec < g.ew;
            const int vy = (int)(((float)er + 0.5f) * inv_t), vx = (int)(((float)ec + 0.5f) * inv_t);
            const int r = er - vy * g.T, c = ec - vx * g.T;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int ty = vy - (q >> 1), tx = vx - (q & 1);
                const int lr = r + (q >> 1) * g.T, lc = c + (q & 1) * g.T;
                const int j = tx - (vxa - 1);
                lo[u][q] = 0;
                cnt[u][q] = 0;
                off[u][q] = lc * g.win + lr;
                if (live && ty >= 0 && tx >= 0 && ty < g.nty && tx < g.ntx && lr < g.win && lc < g.win) {
                    lo[u][q] = rng[ty][j];
                    cnt[u][q] = rng[ty][j + 1] - lo[u][q];
                }
            }
        }
        // every load unconditional (an empty quadrant reads the item's first slot and scales it
        // by 0; a select would be turned back into a branch around the load): a load behind a
        // branch waits for its own round trip before the next is issued
        if (any_slot) {
#pragma unroll
            for (int u = 0; u < FOLD_CELLS; ++u)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const bool on = cnt[u][q] > 0;
                    const int64_t at = on ? (int64_t)lo[u][q] * g.win_stride + off[u][q] : (int64_t)s_first * g.win_stride;
                    const cpx h = slots[at];
                    const real keep = on ? real(1) : real(0);
                    first[u][q] = cpx{h.re * keep, h.im * keep};
                }
        } else {
#pragma unroll
            for (int u = 0; u < FOLD_CELLS; ++u)
#pragma unroll
                for (int q = 0; q < 4; ++q) first[u][q] = cpx{0, 0};
        }
#pragma unroll
        for (int u = 0; u < FOLD_CELLS; ++u) {
            const int e = e0 + u * NT, cc = e >> LOGN, t1 = e & msk, t2 = c0 + cc;
            if (e >= N * CB) break;
            cpx v = cpx{0, 0};
            if (t2 < g.rw) {
                // extended cell of the first row alias
                real ar = real(0), ai = real(0);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (cnt[u][q] > 0) {
                        ar += first[u][q].re;
                        ai += first[u][q].im;
                        for (int k = 1; k < cnt[u][q]; ++k) {
                            const cpx h = slots[(int64_t)(lo[u][q] + k) * g.win_stride + off[u][q]];
                            ar += h.re;
                            ai += h.im;
                        }
                    }
                }
                // pair_sum: the first alias (present when inside the grid), then the second
                const int er = (t1 + g.O) & msk, ec = (t2 + g.O) & msk;
                real hr = real(0), hi = real(0);
                if (ec < g.ew) {
                    if (er < g.eh) {
                        hr += ar;
                        hi += ai;
                    }
                    if (er + g.nf < g.eh) {
                        const cpx b = ext_cell(g, ts, slots, er + g.nf, ec);
                        hr += b.re;
                        hi += b.im;
                    }
                }
                // the Hermitian mirror: extended columns outside this block's tile columns, only
                // near t2 = 0 and t2 = n_f / 2
                const cpx m = alias_from_slots(g, ts, slots, (N - t1) & msk, (N - t2) & msk);
                v = cpx{real(0.5) * (hr + m.re), real(0.5) * (hi - m.im)};
            }
            buf[t1 * CB + cc] = v;
        }
    }
    twr.store(tws);
    __syncthreads();
    fft_lds<LOGN, CB, true>(buf, tws);
    cpx *Ri = R + (int64_t)item * g.r_stride;
    const int nk = g.nk;
    for (int e = tid; e < nk * CB; e += NT) {
        const int a = e / CB, cc = e - (e / CB) * CB;
        if (c0 + cc < g.rw) Ri[(int64_t)a * g.rw + c0 + cc] = buf[((a - nk / 2) & (N - 1)) * CB + cc];
    }
}

// --------------------------------------------------------------- adjoint row pass
template <int LOGN>
__global__ __launch_bounds__(NT) void k_row_inv(Geom g, const cpx *__restrict__ R,
                                                const real *__restrict__ beams,
                                                const real *__restrict__ fscale,
                                                const real *__restrict__ dq,
                                                const cpx *__restrict__ tw, real *__restrict__ gp) {
    constexpr int N = 1 << LOGN;
    __shared__ cpx buf[N];
    __shared__ cpx tws[tw_len<LOGN>()];
    TwStage<LOGN> twr;
    twr.fetch(tw);
    const int tid = threadIdx.x;
    const int item = blockIdx.y;
    const int k = item / g.C, c = item - (item / g.C) * g.C;
    const int a0 = 2 * blockIdx.x;
    const int nk = g.nk;
    const cpx *X = R + (int64_t)item * g.r_stride + (int64_t)a0 * g.rw;
    const cpx *Y = X + g.rw;
    for (int k0 = tid; k0 < N; k0 += COL_LOADS * NT) {
        cpx xv[COL_LOADS], yv[COL_LOADS];
#pragma unroll
        for (int u = 0; u < COL_LOADS; ++u) {
            const int kk = k0 + u * NT;
            if (kk < N) {
                const int src = kk <= N / 2 ? kk : N - kk;
                xv[u] = X[src];
                yv[u] = Y[src];
            }
        }
#pragma unroll
        for (int u = 0; u < COL_LOADS; ++u) {
            const int kk = k0 + u * NT;
            if (kk >= N) break;
            cpx x = xv[u], y = yv[u];
            if (kk <= N / 2) {
                if (kk == 0 || kk == N / 2) { x.im = real(0); y.im = real(0); }
            } else {
                x.im = -x.im;
                y.im = -y.im;
            }
            buf[kk] = cpx{x.re - y.im, x.im + y.re}; // x + i y
        }
    }
    twr.store(tws);
    __syncthreads();
    fft_lds<LOGN, 1, true>(buf, tws);
    const real *A = beams + (int64_t)k * nk * nk;
    real *out = gp + (int64_t)item * nk * nk;
    const real s = fscale[c];
    const real q0 = s * dq[a0], q1 = s * dq[a0 + 1];
    for (int b = tid; b < nk; b += NT) {
        const cpx z = buf[(b - nk / 2) & (N - 1)];
        const int64_t e0 = (int64_t)a0 * nk + b;
        out[e0] = q0 * dq[b] * A[e0] * z.re;
        out[e0 + nk] = q1 * dq[b] * A[e0 + nk] * z.im;
    }
}

// ------------------------------------------------------------------- single dish
__device__ __forceinline__ int floordiv(int a, int b) { return (a >= 0) ? a / b : -((-a + b - 1) / b); }
__device__ __forceinline__ int ceildiv(int a, int b) { return -floordiv(-a, b); }

// U[c][i][q] = sum_j g(o + q S - j) x[c][i][j]   (beam along columns, sampled columns)
__global__ __launch_bounds__(NT) void k_sd_rows(Geom g, const real *__restrict__ sky,
                                                const real *__restrict__ gB, int rb, int sd_n,
                                                int stride, int offset, real *__restrict__ U) {
    const int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x;
    const int64_t tot = (int64_t)g.C * g.N * sd_n;
    if (idx >= tot) return;
    const int q = (int)(idx % sd_n);
    const int64_t ci = idx / sd_n; // c * N + i
    const real *row = sky + ci * g.N;
    const int cen = offset + q * stride;
    real s = real(0);
    const int lo = cen - rb < 0 ? -cen : -rb;
    const int hi = cen + rb >= g.N ? g.N - 1 - cen : rb;
    for (int t = lo; t <= hi; ++t) s += gB[t + rb] * row[cen + t];
    U[idx] = s;
}

// T~[c][p][q] = sum_i g(o + p S - i) U[c][i][q];  E = (T~ - T)/sigma^2;  K partials
__global__ __launch_bounds__(NT) void k_sd_cols(Geom g, const real *__restrict__ U,
                                                const real *__restrict__ gB, int rb, int sd_n,
                                                int stride, int offset, const real *__restrict__ sdmap,
                                                real inv_var, real *__restrict__ E, double *__restrict__ kpart) {
    __shared__ double red[NT / 64];
    const int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x;
    const int64_t tot = (int64_t)g.C * sd_n * sd_n;
    double kk = 0.0;
    if (idx < tot) {
        const int q = (int)(idx % sd_n);
        const int p = (int)((idx / sd_n) % sd_n);
        const int c = (int)(idx / ((int64_t)sd_n * sd_n));
        const int cen = offset + p * stride;
        const int lo = cen - rb < 0 ? -cen : -rb;
        const int hi = cen + rb >= g.N ? g.N - 1 - cen : rb;
        const real *Uc = U + (int64_t)c * g.N * sd_n;
        real s = real(0);
        for (int t = lo; t <= hi; ++t) s += gB[t + rb] * Uc[(int64_t)(cen + t) * sd_n + q];
        const real res = s - sdmap[idx];
        E[idx] = res * inv_var;
        kk = 0.5 * (double)res * (double)res * (double)inv_var;
    }
    for (int m = 32; m >= 1; m >>= 1) kk += __shfl_xor(kk, m, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = kk;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < NT / 64; ++w) s += red[w];
        kpart[blockIdx.x] = s;
    }
}

// V[c][p][j] = sum_q g(o + q S - j) E[c][p][q]: the column half of B^T S^T E, so that the
// sky pass needs only the row sum over the few p whose beam reaches row i
__global__ __launch_bounds__(NT) void k_sd_back(Geom g, const real *__restrict__ E, const real *__restrict__ gB,
                                                int rb, int sd_n, int stride, int offset, real *__restrict__ V) {
    const int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x;
    const int64_t tot = (int64_t)g.C * sd_n * g.N;
    if (idx >= tot) return;
    const int j = (int)(idx % g.N);
    const int64_t cp = idx / g.N; // c * sd_n + p
    const int q0 = max(0, ceildiv(j - rb - offset, stride)), q1 = min(sd_n - 1, floordiv(j + rb - offset, stride));
    const real *Ep = E + cp * sd_n;
    real s = real(0);
    for (int q = q0; q <= q1; ++q) s += gB[offset + q * stride - j + rb] * Ep[q];
    V[idx] = s;
}

// --------------------------------------------------------------------- sky level
static_assert(SKY_T * SKY_T == NT, "one thread per pixel of a sky block");

struct SkyArgs {
    Geom g;
    const real *sky;
    const real *gp;
    const int32_t *cptr;
    const CsrEnt *cent;
    real lambda_r, lambda_s;
    const real *E;
    const real *gB;
    int rb, sd_n, stride, offset;
    real *grad;
    double *rpart;
    int mode;   // SkyMode
    real scale; // gradient multiplier
    real lambda_nu;
    double *npart;
};

constexpr int SKY_LOADS = 8; // CSR entries per lane in flight in k_sky

__global__ __launch_bounds__(NT) void k_sky(SkyArgs a) {
    __shared__ real xs[SKY_T + 4][SKY_T + 5];
    __shared__ real dxs[SKY_T + 2][SKY_T + 3];
    __shared__ double red[NT / 64];
    const Geom &g = a.g;
    const int N = g.N;
    // XCD-aware block order (as col_block) on cubes: each XCD takes a contiguous band of
    // (channel, tile row, tile column) triples, so neighbouring tiles, whose CSR entries
    // gather from the same lines of g', share an L2.  With few channels a band is a strip
    // of one image whose pointing overlap (and so CSR length) varies, which unbalances the
    // XCDs: the launch order is kept there.
    const int nb = (N + SKY_T - 1) / SKY_T;
    const int64_t total = (int64_t)nb * nb * g.C, per = (total + 7) / 8;
    const int64_t bw = g.C >= 8 ? (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3) : (int64_t)blockIdx.x;
    if (bw >= total) return;
    const int bx = (int)(bw % nb), by = (int)((bw / nb) % nb);
    const int c = (int)(bw / ((int64_t)nb * nb));
    const int i0 = by * SKY_T, j0 = bx * SKY_T;
    const int tid = threadIdx.x;
    const int ti = tid / SKY_T, tj = tid - (tid / SKY_T) * SKY_T;
    const real *x = a.sky + (int64_t)c * N * N;
    const bool adjoint_only = a.mode == SKY_ADJOINT, value_only = a.mode == SKY_VALUE;
    const bool reg = (a.lambda_r != real(0)) && !adjoint_only;
    const bool sd = (a.lambda_s != real(0)) && (a.sd_n > 0) && !adjoint_only && !value_only;
    const bool spec = (a.lambda_nu != real(0)) && !adjoint_only && g.C > 1;
    double nloc = 0.0;
    double rloc = 0.0;
    if (reg) {
        for (int e = tid; e < (SKY_T + 4) * (SKY_T + 4); e += NT) {
            const int r = e / (SKY_T + 4), cc = e - (e / (SKY_T + 4)) * (SKY_T + 4);
            const int gi = i0 - 2 + r, gj = j0 - 2 + cc;
            xs[r][cc] = (gi >= 0 && gi < N && gj >= 0 && gj < N) ? x[(int64_t)gi * N + gj] : real(0);
        }
        __syncthreads();
        for (int e = tid; e < (SKY_T + 2) * (SKY_T + 2); e += NT) {
            const int r = e / (SKY_T + 2), cc = e - (e / (SKY_T + 2)) * (SKY_T + 2);
            const int gi = i0 - 1 + r, gj = j0 - 1 + cc;
            real d = real(0);
            if (gi >= 0 && gi < N && gj >= 0 && gj < N)
                d = real(4) * xs[r + 1][cc + 1] - xs[r][cc + 1] - xs[r + 2][cc + 1] - xs[r + 1][cc] - xs[r + 1][cc + 2];
            dxs[r][cc] = d;
        }
        __syncthreads();
    }
    const int i = i0 + ti, j = j0 + tj;
    // spectral term: this pixel in the neighbouring channels
    real xc = real(0), xm = real(0), xp = real(0);
    if (spec && i < N && j < N) {
        const int64_t pix = (int64_t)i * N + j, cs = (int64_t)N * N;
        xc = x[pix];
        if (c > 0) xm = x[pix - cs];
        if (c + 1 < g.C) {
            xp = x[pix + cs];
            const real d = xp - xc;
            nloc = 0.5 * (double)d * (double)d;
        }
    }
    if (value_only) {
        if (reg && i < N && j < N) {
            const real d = dxs[ti + 1][tj + 1];
            rloc = 0.5 * (double)d * (double)d;
        }
    } else if (i < N && j < N) {
        real gsum = real(0);
        const int64_t p = (int64_t)i * N + j;
        const int64_t coff = (int64_t)c * g.nk * g.nk;
        (void)p;
        // this wave's slice: entries lane-contiguous, padded with zero weights
        const int slice = (by * nb + bx) * (NT / 64) + (tid >> 6);
        const int e0 = a.cptr[slice], len = (a.cptr[slice + 1] - e0) >> 6;
        const CsrEnt *en = a.cent + e0 + (tid & 63);
        // SKY_LOADS entries, then their SKY_LOADS gathers, are requested before the first is
        // used; the products are added in entry order
        for (int t0 = 0; t0 < len; t0 += SKY_LOADS) {
            CsrEnt q[SKY_LOADS];
            real v[SKY_LOADS];
#pragma unroll
            for (int u = 0; u < SKY_LOADS; ++u)
                if (t0 + u < len) q[u] = en[(t0 + u) * 64];
#pragma unroll
            for (int u = 0; u < SKY_LOADS; ++u)
                if (t0 + u < len) v[u] = a.gp[(int64_t)q[u].off + coff];
#pragma unroll
            for (int u = 0; u < SKY_LOADS; ++u)
                if (t0 + u < len) gsum += q[u].w * v[u];
        }
        if (reg) {
            const real d = dxs[ti + 1][tj + 1];
            gsum += a.lambda_r * (real(4) * d - dxs[ti][tj + 1] - dxs[ti + 2][tj + 1] - dxs[ti + 1][tj] - dxs[ti + 1][tj + 2]);
            rloc = 0.5 * (double)d * (double)d;
        }
        if (sd) {
            const int S = a.stride, o = a.offset, rb = a.rb;
            const int p0 = max(0, ceildiv(i - rb - o, S)), p1 = min(a.sd_n - 1, floordiv(i + rb - o, S));
            const real *Vc = a.E + (int64_t)c * a.sd_n * N; // V of k_sd_back
            real s = real(0);
            for (int pp = p0; pp <= p1; ++pp) s += a.gB[o + pp * S - i + rb] * Vc[(int64_t)pp * N + j];
            gsum += a.lambda_s * s;
        }
        if (spec) {
            real ds = real(0);
            if (c > 0) ds += xc - xm;
            if (c + 1 < g.C) ds -= xp - xc;
            gsum += a.lambda_nu * ds;
        }
        a.grad[(int64_t)c * N * N + p] = a.scale == real(1) ? gsum : a.scale * gsum;
    }
    if (!adjoint_only) {
        for (int m = 32; m >= 1; m >>= 1) rloc += __shfl_xor(rloc, m, 64);
        if ((tid & 63) == 0) red[tid >> 6] = rloc;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int w = 0; w < NT / 64; ++w) s += red[w];
            a.rpart[bw] = s;
        }
        if (spec) {
            __syncthreads(); // red is reused
            for (int m = 32; m >= 1; m >>= 1) nloc += __shfl_xor(nloc, m, 64);
            if ((tid & 63) == 0) red[tid >> 6] = nloc;
            __syncthreads();
            if (tid == 0) {
                double s = 0.0;
                for (int w = 0; w < NT / 64; ++w) s += red[w];
                a.npart[bw] = s;
            }
        }
    }
}

// ---------------------------------------------------------------------- reductions
// out[b] = sum of in[b * per .. (b + 1) * per) (fixed order: strided per thread, then tree)
__global__ __launch_bounds__(NT) void k_partial_sums(const double *__restrict__ in, int n, int per,
                                                     double *__restrict__ out) {
    __shared__ double red[NT / 64];
    const int b0 = blockIdx.x * per, b1 = min(n, b0 + per);
    double v = 0.0;
    int i = b0 + threadIdx.x;
    for (; i + 7 * NT < b1; i += 8 * NT) {
        double t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = in[i + u * NT];
#pragma unroll
        for (int u = 0; u < 8; ++u) v += t[u];
    }
    for (; i < b1; i += NT) v += in[i];
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < NT / 64; ++w) s += red[w];
        out[blockIdx.x] = s;
    }
}

constexpr int NT_FINAL = 1024;
constexpr int FINAL_PER = 1024; // work-item partials per pre-reduction block
__global__ __launch_bounds__(NT_FINAL) void k_final(const double *__restrict__ jpart, int nj,
                                                    const double *__restrict__ rpart, int nr,
                                                    const double *__restrict__ kpart, int nkp,
                                                    const double *__restrict__ npart, int nnp,
                                                    double lambda_r, double lambda_s, double lambda_nu,
                                                    double *terms, double *terms_user) {
    __shared__ double sh[4][NT_FINAL / 64];
    const int tid = threadIdx.x;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    // each thread sums its strided entries in index order; 8 loads are issued before they
    // are added, so their latencies overlap instead of chaining
    auto strided_sum = [&](const double *__restrict__ p, int n, double &acc) {
        int i = tid;
        for (; i + 7 * NT_FINAL < n; i += 8 * NT_FINAL) {
            double t[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) t[u] = p[i + u * NT_FINAL];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc += t[u];
        }
        for (; i < n; i += NT_FINAL) acc += p[i];
    };
    strided_sum(jpart, nj, v[0]);
    strided_sum(rpart, nr, v[1]);
    strided_sum(kpart, nkp, v[2]);
    strided_sum(npart, nnp, v[3]);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        for (int m = 32; m >= 1; m >>= 1) v[q] += __shfl_xor(v[q], m, 64);
        if ((tid & 63) == 0) sh[q][tid >> 6] = v[q];
    }
    __syncthreads();
    if (tid == 0) {
        double Q = 0.0, R = 0.0, K = 0.0, Nu = 0.0;
        for (int w = 0; w < NT_FINAL / 64; ++w) {
            Q += sh[0][w];
            R += sh[1][w];
            K += sh[2][w];
            Nu += sh[3][w];
        }
        double qt = Q + lambda_s * K + lambda_r * R;
        if (lambda_nu != 0.0) qt += lambda_nu * Nu;
        const double t5[5] = {qt, Q, K, R, Nu};
        for (int q = 0; q < 5; ++q) terms[q] = t5[q];
        if (terms_user)
            for (int q = 0; q < 4; ++q) terms_user[q] = t5[q];
    }
}

__global__ __launch_bounds__(NT) void k_zero(uint32_t *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) p[i] = 0u;
}

// ------------------------------------------------------------------------ feathering
// App. B: out = F^-1[B F[sd] + (1 - B) F[int]] = int + F^-1[B F[sd - int]] (B real and even),
// per channel of n x n maps: a real row FFT of the difference (two rows packed in one complex
// transform, half spectrum kept), a column FFT, the Gaussian transfer function
// B(k) = exp(-2 pi^2 sigma^2 |k|^2), the inverse column FFT, and the inverse row FFT, added to
// the interferometric map with the 1 / n^2 of the unscaled transform pair.  Work: the
// half-spectra [C][n][n/2 + 1] complex.  Twiddles are formed in LDS from FP64 sincospi.
template <int LOGN> __device__ __forceinline__ void tw_fill(cpx *tws) {
    constexpr int N = 1 << LOGN;
    for (int t = threadIdx.x; t < tw_len<LOGN>(); t += NT) {
        double sv, cv;
        sincospi(-2.0 * (double)t / (double)N, &sv, &cv);
        tws[t] = cpx{(real)cv, (real)sv};
    }
}

template <int LOGN>
__global__ __launch_bounds__(NT) void k_feather_rows(const real *__restrict__ interf, const real *__restrict__ sd,
                                                     cpx *__restrict__ work) {
    constexpr int N = 1 << LOGN, RW = N / 2 + 1;
    __shared__ cpx buf[N];
    __shared__ cpx tws[tw_len<LOGN>()];
    const int c = blockIdx.y, a0 = 2 * blockIdx.x;
    const int64_t base = ((int64_t)c * N + a0) * N;
    for (int b = threadIdx.x; b < N; b += NT)
        buf[b] = cpx{sd[base + b] - interf[base + b], sd[base + N + b] - interf[base + N + b]};
    tw_fill<LOGN>(tws);
    __syncthreads();
    fft_lds<LOGN, 1, false>(buf, tws);
    cpx *W0 = work + ((int64_t)c * N + a0) * RW, *W1 = W0 + RW;
    for (int kk = threadIdx.x; kk < RW; kk += NT) {
        const cpx z = buf[kk], zm = buf[(N - kk) & (N - 1)];
        W0[kk] = cpx{real(0.5) * (z.re + zm.re), real(0.5) * (z.im - zm.im)};
        W1[kk] = cpx{real(0.5) * (z.im + zm.im), real(0.5) * (zm.re - z.re)};
    }
}

template <int LOGN, int CB>
__global__ __launch_bounds__(NT) void k_feather_cols(cpx *__restrict__ work, double knorm2) {
    constexpr int N = 1 << LOGN, RW = N / 2 + 1;
    __shared__ cpx buf[CB * N];
    __shared__ cpx tws[tw_len<LOGN>()];
    const int c = blockIdx.y, c0 = blockIdx.x * CB;
    cpx *Wc = work + (int64_t)c * N * RW;
    for (int e = threadIdx.x; e < N * CB; e += NT) {
        const int q = e / CB, cc = e - q * CB;
        buf[q * CB + cc] = c0 + cc < RW ? Wc[(int64_t)q * RW + c0 + cc] : cpx{0, 0};
    }
    tw_fill<LOGN>(tws);
    __syncthreads();
    fft_lds<LOGN, CB, false>(buf, tws);
    // B(k) with k^2 = (p^2 + q^2) / (n delta)^2; knorm2 = 2 pi^2 sigma^2 / (n delta)^2
    for (int e = threadIdx.x; e < N * CB; e += NT) {
        const int q = e / CB, cc = e - q * CB;
        const int qs = q < N / 2 ? q : q - N, ps = c0 + cc;
        const real bk = (real)exp(-knorm2 * ((double)ps * ps + (double)qs * qs));
        buf[e] = cpx{bk * buf[e].re, bk * buf[e].im};
    }
    __syncthreads();
    fft_lds<LOGN, CB, true>(buf, tws);
    for (int e = threadIdx.x; e < N * CB; e += NT) {
        const int q = e / CB, cc = e - q * CB;
        if (c0 + cc < RW) Wc[(int64_t)q * RW + c0 + cc] = buf[q * CB + cc];
    }
}

template <int LOGN>
__global__ __launch_bounds__(NT) void k_feather_rows_inv(const real *__restrict__ interf, const cpx *__restrict__ work,
                                                         real *__restrict__ out) {
    constexpr int N = 1 << LOGN, RW = N / 2 + 1;
    __shared__ cpx buf[N];
    __shared__ cpx tws[tw_len<LOGN>()];
    const int c = blockIdx.y, a0 = 2 * blockIdx.x;
    const cpx *X = work + ((int64_t)c * N + a0) * RW, *Y = X + RW;
    for (int kk = threadIdx.x; kk < N; kk += NT) {
        const int src = kk <= N / 2 ? kk : N - kk;
        cpx x = X[src], y = Y[src];
        if (kk > N / 2) {
            x.im = -x.im;
            y.im = -y.im;
        }
        buf[kk] = cpx{x.re - y.im, x.im + y.re}; // x + i y
    }
    tw_fill<LOGN>(tws);
    __syncthreads();
    fft_lds<LOGN, 1, true>(buf, tws);
    const real sc = real(1) / ((real)N * (real)N);
    const int64_t base = ((int64_t)c * N + a0) * N;
    for (int b = threadIdx.x; b < N; b += NT) {
        out[base + b] = interf[base + b] + sc * buf[b].re;
        out[base + N + b] = interf[base + N + b] + sc * buf[b].im;
    }
}

// ===================================================================== launchers

#define IVX_LOGN_SWITCH(LOGN_VAR, ...)                       \
    switch (LOGN_VAR) {                                      \
    case 6: { constexpr int L = 6; __VA_ARGS__; } break;     \
    case 7: { constexpr int L = 7; __VA_ARGS__; } break;     \
    case 8: { constexpr int L = 8; __VA_ARGS__; } break;     \
    case 9: { constexpr int L = 9; __VA_ARGS__; } break;     \
    case 10: { constexpr int L = 10; __VA_ARGS__; } break;   \
    case 11: { constexpr int L = 11; __VA_ARGS__; } break;   \
    default: return hipErrorInvalidValue;                    \
    }

static int n_items(const Geom &g) { return g.C * g.P; }

hipError_t launch_image_rows(const Geom &g, const real *sky, const real *beams, const real *interp,
                             const real *fscale, const real *dq, const cpx *tw, cpx *R, hipStream_t st) {
    dim3 grid(g.nk / 2, n_items(g));
    IVX_LOGN_SWITCH(g.logn, (k_image_rows<L><<<grid, NT, 0, st>>>(g, sky, beams, interp, fscale, dq, tw, R)));
    return hipGetLastError();
}

// Columns per block: col_batch's width (wider blocks write longer row segments), but narrow
// enough that the launch has about two blocks per compute unit.
template <int LOGN> static int pick_cb(const Geom &g) {
    int cb = col_batch<LOGN>();
    while (cb > 1 && (int64_t)((g.rw + cb - 1) / cb) * n_items(g) < 512) cb >>= 1;
    return cb;
}

// Launch size of a column pass: (item, column group) pairs rounded up to a multiple of 8
// (see col_block).
static dim3 col_grid(const Geom &g, int cb) {
    const int64_t total = (int64_t)((g.rw + cb - 1) / cb) * n_items(g);
    return dim3((unsigned)(8 * ((total + 7) / 8)));
}

#define IVX_CB_SWITCH(CBV, ...)                                                   \
    switch (CBV) {                                                                \
    case 1: { constexpr int B = 1; __VA_ARGS__; } break;                          \
    case 2: { constexpr int B = 2 <= col_batch<L>() ? 2 : 1; __VA_ARGS__; } break;   \
    case 4: { constexpr int B = 4 <= col_batch<L>() ? 4 : 1; __VA_ARGS__; } break;   \
    case 8: { constexpr int B = 8 <= col_batch<L>() ? 8 : 1; __VA_ARGS__; } break;   \
    default: { constexpr int B = 16 <= col_batch<L>() ? 16 : 1; __VA_ARGS__; } break; \
    }

hipError_t launch_col_fwd(const Geom &g, const cpx *R, const cpx *tw, cpx *ext, hipStream_t st) {
    IVX_LOGN_SWITCH(g.logn, {
        const int cb = pick_cb<L>(g);
        IVX_CB_SWITCH(cb, {
            k_col_fwd<L, B><<<col_grid(g, B), NT, 0, st>>>(g, R, tw, ext);
        });
    });
    return hipGetLastError();
}

hipError_t launch_col_inv(const Geom &g, const cpx *E, const cpx *tw, cpx *R, hipStream_t st) {
    IVX_LOGN_SWITCH(g.logn, {
        const int cb = pick_cb<L>(g);
        IVX_CB_SWITCH(cb, {
            k_col_inv<L, B><<<col_grid(g, B), NT, 0, st>>>(g, E, tw, R);
        });
    });
    return hipGetLastError();
}

// The fused pass has one block per (item, column group): worth it once that fills the chip
// several times over (the two-kernel fold has more, smaller blocks for few-item plans).
constexpr int64_t FUSED_FOLD_MIN_BLOCKS = 2048;

bool fold_fusable(const Geom &g) { return g.eh <= 2 * g.nf && g.ew <= g.nf; }

bool fold_fusion_pays(const Geom &g) {
    const int64_t ngrp = (g.rw + IVX_FOLD_CB - 1) / IVX_FOLD_CB;
    return ngrp * g.C * g.P >= FUSED_FOLD_MIN_BLOCKS;
}

hipError_t launch_col_inv_slots(const Geom &g, const int32_t *tslot, const cpx *slots, const cpx *tw, cpx *R,
                                hipStream_t st) {
    if (!fold_fusable(g)) return hipErrorInvalidValue;
    IVX_LOGN_SWITCH(g.logn, {
        const int cb = std::min(pick_cb<L>(g), IVX_FOLD_CB);
        IVX_CB_SWITCH(cb, {
            k_col_inv_slots<L, B><<<col_grid(g, B), NT, 0, st>>>(g, tslot, slots, tw, R);
        });
    });
    return hipGetLastError();
}

hipError_t launch_fold(const Geom &g, const int32_t *tslot, const cpx *slots, cpx *ext, hipStream_t st,
                       const uint8_t *sact) {
    const int tpb = g.T * g.T >= NT ? 1 : NT / (g.T * g.T);
    const int nvt = (g.nty + 1) * (g.ntx + 1);
    k_ext_sum<<<dim3((unsigned)((nvt + tpb - 1) / tpb), n_items(g)), NT, 0, st>>>(g, tpb, tslot, slots, sact, ext);
    return hipGetLastError();
}

hipError_t launch_row_inv(const Geom &g, const cpx *R, const real *beams, const real *fscale,
                          const real *dq, const cpx *tw, real *gp, hipStream_t st) {
    dim3 grid(g.nk / 2, n_items(g));
    IVX_LOGN_SWITCH(g.logn, (k_row_inv<L><<<grid, NT, 0, st>>>(g, R, beams, fscale, dq, tw, gp)));
    return hipGetLastError();
}

size_t grid_lds_bytes(const Geom &g, int nwave, int lanes) {
    if (lanes == GRID_MFMA_LANES) return 0;
    return (size_t)(1 + grid_groups_per_wave(g.W, lanes) * nwave) * g.win * g.ldw * sizeof(cpx);
}

template <int W, int G, int VPI>
static hipError_t launch_grid_wg(int mode, const GridArgs &a, int n_work, hipStream_t st) {
    const size_t wsz = (size_t)a.g.win * a.g.ldw * sizeof(cpx);
    const int threads = 64 * a.nwave;
    const int ng = (64 / G) * a.nwave;
    const unsigned gx = (unsigned)n_work < GRID_ROW ? (unsigned)n_work : GRID_ROW;
    const dim3 grid(gx, (unsigned)((n_work + gx - 1) / gx));
    switch (mode) {
    case MODE_OBJ: k_grid<W, MODE_OBJ, G, VPI><<<grid, threads, (1 + ng) * wsz, st>>>(a); break;
    case MODE_FWD: k_grid<W, MODE_FWD, G, VPI><<<grid, threads, wsz, st>>>(a); break;
    case MODE_VAL: k_grid<W, MODE_VAL, G, VPI><<<grid, threads, wsz, st>>>(a); break;
    default: k_grid<W, MODE_ADJ, G, VPI><<<grid, threads, ng * wsz, st>>>(a); break;
    }
    return hipGetLastError();
}

template <int W, int G, int VPI> static hipError_t prepare_grid_wg(const Geom &g, int nwave) {
    // raise the dynamic-LDS limit of the three modes ahead of any stream capture
    const size_t wsz = (size_t)g.win * g.ldw * sizeof(cpx);
    const int ng = (64 / G) * nwave;
    hipError_t e;
    if ((e = hipFuncSetAttribute((const void *)k_grid<W, MODE_OBJ, G, VPI>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)((1 + ng) * wsz))) != hipSuccess)
        return e;
    if ((e = hipFuncSetAttribute((const void *)k_grid<W, MODE_FWD, G, VPI>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)wsz)) != hipSuccess)
        return e;
    if ((e = hipFuncSetAttribute((const void *)k_grid<W, MODE_VAL, G, VPI>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)wsz)) != hipSuccess)
        return e;
    return hipFuncSetAttribute((const void *)k_grid<W, MODE_ADJ, G, VPI>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(ng * wsz));
}

template <int W, int G>
static hipError_t dispatch_wg(bool prepare, int vpi, int mode, const GridArgs &a, int n_work, hipStream_t st) {
    if (vpi == 2) return prepare ? prepare_grid_wg<W, G, 2>(a.g, a.nwave) : launch_grid_wg<W, G, 2>(mode, a, n_work, st);
    return prepare ? prepare_grid_wg<W, G, 1>(a.g, a.nwave) : launch_grid_wg<W, G, 1>(mode, a, n_work, st);
}

// variant = 10 * lanes + visibilities per group per iteration (81, 82, 161, 162)
template <int W>
static hipError_t dispatch_w(bool prepare, int variant, int mode, const GridArgs &a, int n_work, hipStream_t st) {
    const int lanes = variant / 10, vpi = variant % 10;
    if constexpr (W <= 8) {
        if (lanes == 8) return dispatch_wg<W, 8>(prepare, vpi, mode, a, n_work, st);
    }
    return dispatch_wg<W, 16>(prepare, vpi, mode, a, n_work, st);
}

static hipError_t dispatch(bool prepare, int variant, int mode, const GridArgs &a, int n_work, hipStream_t st) {
    switch (a.g.W) {
    case 4: return dispatch_w<4>(prepare, variant, mode, a, n_work, st);
    case 5: return dispatch_w<5>(prepare, variant, mode, a, n_work, st);
    case 6: return dispatch_w<6>(prepare, variant, mode, a, n_work, st);
    case 7: return dispatch_w<7>(prepare, variant, mode, a, n_work, st);
    case 8: return dispatch_w<8>(prepare, variant, mode, a, n_work, st);
    case 9: return dispatch_w<9>(prepare, variant, mode, a, n_work, st);
    case 10: return dispatch_w<10>(prepare, variant, mode, a, n_work, st);
    case 11: return dispatch_w<11>(prepare, variant, mode, a, n_work, st);
    case 12: return dispatch_w<12>(prepare, variant, mode, a, n_work, st);
    case 13: return dispatch_w<13>(prepare, variant, mode, a, n_work, st);
    case 14: return dispatch_w<14>(prepare, variant, mode, a, n_work, st);
    case 15: return dispatch_w<15>(prepare, variant, mode, a, n_work, st);
    case 16: return dispatch_w<16>(prepare, variant, mode, a, n_work, st);
    default: return hipErrorInvalidValue;
    }
}

#ifndef IVX_REAL_DOUBLE
template <int KW, int OCC> void launch_gridmx_occ(int mode, dim3 grid, const GridArgs &a, hipStream_t st) {
    switch (mode) {
    case MODE_OBJ: k_gridmx<MODE_OBJ, KW, OCC><<<grid, 64, 0, st>>>(a); break;
    case MODE_FWD: k_gridmx<MODE_FWD, KW, OCC><<<grid, 64, 0, st>>>(a); break;
    case MODE_VAL: k_gridmx<MODE_VAL, KW, OCC><<<grid, 64, 0, st>>>(a); break;
    case MODE_WFWD: k_gridmx<MODE_WFWD, KW, OCC><<<grid, 64, 0, st>>>(a); break;
    case MODE_WADJ: k_gridmx<MODE_WADJ, KW, OCC><<<grid, 64, 0, st>>>(a); break;
    default: k_gridmx<MODE_ADJ, KW, OCC><<<grid, 64, 0, st>>>(a); break;
    }
}

// Work items beyond which the 7-waves-per-SIMD build is used (about four rounds of waves
// on 1,024 SIMDs).
constexpr int64_t GRIDMX_OCC7_ITEMS = 32768;

template <int KW> void launch_gridmx(int mode, dim3 grid, const GridArgs &a, int occ, hipStream_t st) {
    if (occ == GRIDMX_OCC_AUTO) occ = a.n_work >= GRIDMX_OCC7_ITEMS ? 7 : 6;
    if (occ == 7) launch_gridmx_occ<KW, 7>(mode, grid, a, st);
    else launch_gridmx_occ<KW, 6>(mode, grid, a, st);
}
#endif

// w-plane passes: 16-lane groups, one visibility per group per iteration, any kernel width.
template <int W> static hipError_t wgrid_w(bool prepare, int mode, const GridArgs &a, int n_work, hipStream_t st) {
    const size_t wsz = (size_t)a.g.win * a.g.ldw * sizeof(cpx);
    const int ng = 4 * a.nwave;
    if (prepare) {
        hipError_t e = hipFuncSetAttribute((const void *)k_grid<W, MODE_WFWD, 16, 1>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)wsz);
        if (e != hipSuccess) return e;
        return hipFuncSetAttribute((const void *)k_grid<W, MODE_WADJ, 16, 1>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)(ng * wsz));
    }
    const unsigned gx = (unsigned)n_work < GRID_ROW ? (unsigned)n_work : GRID_ROW;
    const dim3 grid(gx, (unsigned)((n_work + gx - 1) / gx));
    if (mode == MODE_WFWD) k_grid<W, MODE_WFWD, 16, 1><<<grid, 64 * a.nwave, wsz, st>>>(a);
    else k_grid<W, MODE_WADJ, 16, 1><<<grid, 64 * a.nwave, ng * wsz, st>>>(a);
    return hipGetLastError();
}

static hipError_t wgrid_dispatch(bool prepare, int mode, const GridArgs &a, int n_work, hipStream_t st) {
    switch (a.g.W) {
    case 4: return wgrid_w<4>(prepare, mode, a, n_work, st);
    case 5: return wgrid_w<5>(prepare, mode, a, n_work, st);
    case 6: return wgrid_w<6>(prepare, mode, a, n_work, st);
    case 7: return wgrid_w<7>(prepare, mode, a, n_work, st);
    case 8: return wgrid_w<8>(prepare, mode, a, n_work, st);
    case 9: return wgrid_w<9>(prepare, mode, a, n_work, st);
    case 10: return wgrid_w<10>(prepare, mode, a, n_work, st);
    case 11: return wgrid_w<11>(prepare, mode, a, n_work, st);
    case 12: return wgrid_w<12>(prepare, mode, a, n_work, st);
    case 13: return wgrid_w<13>(prepare, mode, a, n_work, st);
    case 14: return wgrid_w<14>(prepare, mode, a, n_work, st);
    case 15: return wgrid_w<15>(prepare, mode, a, n_work, st);
    case 16: return wgrid_w<16>(prepare, mode, a, n_work, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t prepare_wgrid(const Geom &g, int nwave) {
    GridArgs a{};
    a.g = g;
    a.nwave = nwave;
    return wgrid_dispatch(true, MODE_WFWD, a, 0, nullptr);
}

hipError_t launch_wgrid(int mode, const Geom &g, const WorkItem *work, int n_work, const VisCoord *crd,
                        const cpx *ext, cpx *slots, const WPlane &wp, int nwave, int variant, int occupancy,
                        hipStream_t st) {
    if (mode != MODE_WFWD && mode != MODE_WADJ) return hipErrorInvalidValue;
    if (n_work <= 0) return hipSuccess;
    if (nwave < 1 || nwave > NT / 64 || wp.W < 2 || wp.W > 16) return hipErrorInvalidValue;
    if (!(occupancy == GRIDMX_OCC_AUTO || occupancy == 6 || occupancy == 7)) return hipErrorInvalidValue;
    GridArgs a{};
    a.g = g;
    a.work = work;
    a.crd = crd;
    a.ext = ext;
    a.slots = slots;
    a.nwave = nwave;
    a.n_work = n_work;
    a.wz = wp.wz;
    a.wacc = wp.acc;
    a.wq = wp.q;
    a.wplane = wp.plane;
    a.wW = wp.W;
    a.wcnt = wp.cnt;
    a.wncnt = wp.ncnt;
    a.wsact = mode == MODE_WADJ ? wp.sact : nullptr;
#ifdef IVX_REAL_DOUBLE
    a.wbeta2 = wp.beta;
#else
    a.wbeta2 = (real)(wp.beta * 1.4426950408889634);
#endif
    if (variant == GRID_MFMA_VARIANT) {
#ifdef IVX_REAL_DOUBLE
        return hipErrorInvalidValue;
#else
        if (g.win > 16) return hipErrorInvalidValue;
        const unsigned gx = (unsigned)n_work < GRID_ROW ? (unsigned)n_work : GRID_ROW;
        const dim3 grid(gx, (unsigned)((n_work + gx - 1) / gx));
        switch (g.W) {
        case 7: launch_gridmx<7>(mode, grid, a, occupancy, st); break;
        case 8: launch_gridmx<8>(mode, grid, a, occupancy, st); break;
        default: launch_gridmx<0>(mode, grid, a, occupancy, st); break;
        }
        return hipGetLastError();
#endif
    }
    return wgrid_dispatch(false, mode, a, n_work, st);
}

hipError_t prepare_grid(const Geom &g, int nwave, int variant) {
    if (variant == GRID_MFMA_VARIANT) return hipSuccess; // static LDS only
    GridArgs a{};
    a.g = g;
    a.nwave = nwave;
    return dispatch(true, variant, MODE_OBJ, a, 0, nullptr);
}


hipError_t launch_grid(int mode, const Geom &g, const WorkItem *work, int n_work, const VisCoord *crd,
                       const cpx *vis, const real *wgt, const int32_t *perm, const int64_t *boff, const cpx *ext,
                       cpx *slots, double *jpart, const cpx *caller_in, cpx *caller_out, int nwave, int variant,
                       int occupancy, hipStream_t st, bool unweighted) {
    if (!(occupancy == GRIDMX_OCC_AUTO || occupancy == 6 || occupancy == 7)) return hipErrorInvalidValue;
    if (n_work <= 0) return hipSuccess;
    if (nwave < 1 || nwave > NT / 64) return hipErrorInvalidValue;
    GridArgs a{g, work, crd, vis, wgt, perm, boff, ext, slots, jpart, caller_in, caller_out, nwave, n_work,
               unweighted ? 1 : 0};
    if (variant == GRID_MFMA_VARIANT) {
#ifdef IVX_REAL_DOUBLE
        return hipErrorInvalidValue;
#else
        if (g.win > 16) return hipErrorInvalidValue;
        const unsigned gx = (unsigned)n_work < GRID_ROW ? (unsigned)n_work : GRID_ROW;
        const dim3 grid(gx, (unsigned)((n_work + gx - 1) / gx));
        switch (g.W) {
        case 7: launch_gridmx<7>(mode, grid, a, occupancy, st); break;
        case 8: launch_gridmx<8>(mode, grid, a, occupancy, st); break;
        default: launch_gridmx<0>(mode, grid, a, occupancy, st); break;
        }
        return hipGetLastError();
#endif
    }
    return dispatch(false, variant, mode, a, n_work, st);
}

hipError_t launch_sd_rows(const Geom &g, const real *sky, const real *gB, int rb, int sd_n, int stride,
                          int offset, real *U, hipStream_t st) {
    const int64_t tot = (int64_t)g.C * g.N * sd_n;
    k_sd_rows<<<(unsigned)((tot + NT - 1) / NT), NT, 0, st>>>(g, sky, gB, rb, sd_n, stride, offset, U);
    return hipGetLastError();
}

hipError_t launch_sd_cols(const Geom &g, const real *U, const real *gB, int rb, int sd_n, int stride,
                          int offset, const real *sdmap, real inv_var, real *E, double *kpart, hipStream_t st) {
    const int64_t tot = (int64_t)g.C * sd_n * sd_n;
    k_sd_cols<<<(unsigned)((tot + NT - 1) / NT), NT, 0, st>>>(g, U, gB, rb, sd_n, stride, offset, sdmap,
                                                              inv_var, E, kpart);
    return hipGetLastError();
}

hipError_t launch_sd_back(const Geom &g, const real *E, const real *gB, int rb, int sd_n, int stride, int offset,
                          real *V, hipStream_t st) {
    const int64_t tot = (int64_t)g.C * sd_n * g.N;
    k_sd_back<<<(unsigned)((tot + NT - 1) / NT), NT, 0, st>>>(g, E, gB, rb, sd_n, stride, offset, V);
    return hipGetLastError();
}

int sky_blocks(const Geom &g) {
    const int nb = (g.N + SKY_T - 1) / SKY_T;
    return nb * nb * g.C;
}

hipError_t launch_sky(const Geom &g, const real *sky, const real *gp, const int32_t *cptr, const CsrEnt *cent,
                      real lambda_r, real lambda_s, const real *E, const real *gB, int rb, int sd_n, int stride,
                      int offset, real *grad, double *rpart, int mode, real scale, hipStream_t st, real lambda_nu,
                      double *npart) {
    const int nb = (g.N + SKY_T - 1) / SKY_T;
    if (lambda_nu != real(0) && !npart) return hipErrorInvalidValue;
    SkyArgs a{g,    sky,  gp,    cptr,  cent,      lambda_r, lambda_s, E, gB, rb, sd_n, stride, offset, grad, rpart,
              mode, scale, lambda_nu, npart};
    const int64_t total = (int64_t)nb * nb * g.C;
    k_sky<<<dim3((unsigned)(8 * ((total + 7) / 8))), NT, 0, st>>>(a);
    return hipGetLastError();
}

int final_scratch(int nj) { return nj > 32 * FINAL_PER ? (nj + FINAL_PER - 1) / FINAL_PER : 0; }

hipError_t launch_final(const double *jpart, int nj, double *scratch, const double *rpart, int nr,
                        const double *kpart, int nkp, const double *npart, int nnp, double lambda_r,
                        double lambda_s, double lambda_nu, double *terms, double *terms_user, hipStream_t st) {
    const int nb = final_scratch(nj);
    if (nb > 0) {
        // long per-work-item lists (large mosaics): pre-reduce in fixed blocks first
        k_partial_sums<<<nb, NT, 0, st>>>(jpart, nj, FINAL_PER, scratch);
        jpart = scratch;
        nj = nb;
    }
    k_final<<<1, NT_FINAL, 0, st>>>(jpart, nj, rpart, nr, kpart, nkp, npart, nnp, lambda_r, lambda_s, lambda_nu, terms,
                                    terms_user);
    return hipGetLastError();
}

int64_t feather_work_bytes(int n_chan, int n) { return (int64_t)n_chan * n * (n / 2 + 1) * (int64_t)sizeof(cpx); }

hipError_t launch_feather(int n_chan, int n, double delta, double theta, const real *interf, const real *sd, real *out,
                          void *work, hipStream_t st) {
    int logn = 0;
    while ((1 << logn) < n) ++logn;
    cpx *w = static_cast<cpx *>(work);
    const double sigma = theta / (2.0 * sqrt(2.0 * log(2.0)));
    const double knorm2 = 2.0 * M_PI * M_PI * sigma * sigma / ((double)n * delta * (double)n * delta);
    const int rw = n / 2 + 1;
    IVX_LOGN_SWITCH(logn, {
        constexpr int CB = col_batch<L>();
        k_feather_rows<L><<<dim3(n / 2, n_chan), NT, 0, st>>>(interf, sd, w);
        k_feather_cols<L, CB><<<dim3((rw + CB - 1) / CB, n_chan), NT, 0, st>>>(w, knorm2);
        k_feather_rows_inv<L><<<dim3(n / 2, n_chan), NT, 0, st>>>(interf, w, out);
    });
    return hipGetLastError();
}

hipError_t launch_zero(void *p, int64_t bytes, hipStream_t st) {
    if (bytes <= 0) return hipSuccess;
    if (bytes % 4) return hipErrorInvalidValue;
    const int64_t n = bytes / 4;
    int64_t blocks = (n + NT - 1) / NT;
    if (blocks > 4096) blocks = 4096;
    k_zero<<<(unsigned)blocks, NT, 0, st>>>((uint32_t *)p, n);
    return hipGetLastError();
}

} // namespace ivx
