// Positivity-bounded L-BFGS-B on the device (Sect. 3.4, Eq. L-BFGS-B).
//
// The iterate, gradient and correction pairs live in device memory in FP64; every
// length-n operation is a kernel here, and the host keeps only the O(m^2) compact-form
// matrices and the line-search state, reading back a handful of scalars per step.
//
// Generalized Cauchy point without a sequential walk: the method visits the breakpoints
// t_i = x_i / g_i (g_i > 0) in increasing order and updates, at breakpoint b,
//     p <- p + g_b w_b,   c <- c + dt p,
//     f'' <- f'' - theta g_b^2 - 2 g_b w_b.M p - g_b^2 w_b.M w_b,
//     f'  <- f' + dt f'' + g_b^2 + theta g_b z_b - g_b w_b.M c,
// stopping at the first breakpoint whose segment contains the minimiser -f'/f''.  With
// q_j = g_b w_b these are prefix sums: P_j = p_0 + sum_{i<j} q_i, C_j = sum_{i<j} dt_i P_i,
// f''_j = f''_0 - sum_{i<j} (theta g_i^2 + 2 q_i.M P_i + q_i.M q_i),
// f'_j = f'_0 + sum_{i<j} (dt_i f''_i + g_i^2 + theta g_i z_i - q_i.M C_{i+1}),
// so after a device radix sort of the breakpoints the whole walk is five scans and one
// parallel search for the first j with -f'_j / f''_j < dt_j.
#include "ivx_internal.hpp"
#include "ivx_lbfgsb.h"


#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

namespace ivx {
ivx_status set_error(ivx_status s, const std::string &msg);
int64_t plan_sky_count(const ivx_plan *p);
} // namespace ivx

using namespace ivx;

namespace {

constexpr int NT = 256;
constexpr int MAXM = IVX_LBFGSB_MAX_M;
constexpr int MAXD = 2 * MAXM;
constexpr int MAXNV = 4 + 3 * MAXM + 2; // reduced quantities of one kernel
constexpr int RBLK = 512;               // blocks of a reduction grid
constexpr int SEG = 4 * NT;             // elements per block of a scan
constexpr double EPS = 2.220446049250313e-16;
constexpr double INF = std::numeric_limits<double>::infinity();

struct Slots {
    int idx[MAXM]; // chronological order, oldest first
    int k;
    int pad;
};
struct Vec {
    double v[MAXD];
};
struct Half {
    double v[MAXM];
};
// Fixed layouts of the reduced quantities (entries past the stored pairs stay zero).
constexpr int CP_NS = 3 + 2 * MAXM;      // k_cp_init: d.d, #breakpoints, #fixed, Y.d, S.d | t_min
constexpr int UP_NS = 4 + 3 * MAXM;      // k_update: s.y, y.y, g.s, s.s, s.Y, S.y, s.S | -pg
constexpr int SCAL = 2048;               // doubles of the device/host scalar exchange buffers
constexpr int OFF = 8;                   // reductions land at scal[OFF..]; scal[0..4) = terms
constexpr int SEL_OUT = SCAL - 1;        // the breakpoint prefix length (k_cp_select)
constexpr int FLAG = SCAL - 2;           // the sequence number of the last published result
// the host's M for the next walk (k_cp_init moves it to Mdev), after the subspace results
constexpr int MOFF = (OFF + MAXD + MAXD * (MAXD + 1) / 2 + 63) / 64 * 64;
constexpr int PART_R = RBLK * MAXD * (MAXD + 1) / 2; // W^T r partials beside the Gram matrix's
static_assert(OFF + MAXD + MAXD * (MAXD + 1) / 2 <= MOFF && MOFF + MAXD * MAXD <= FLAG,
              "the subspace results, M and the prefix length fit the exchange buffer apart");

// ---------------------------------------------------------------- reductions
// Each thread holds nv partials: entries [0, nsum) are sums, the rest minima.  Wave
// shuffles, then the block's waves in order, one row of `part` per block; finish_sums
// adds the rows in block order.  The shuffle steps run over all quantities at once: the
// exchanges of one step are independent and in flight together, where a chain per
// quantity paid one LDS round trip per step and quantity (216 for 36 quantities).  Each
// quantity is combined in the same order either way.  acc is overwritten.
template <int NV>
__device__ __forceinline__ void block_reduce(double (&acc)[NV], int nv, int nsum, double *__restrict__ part) {
    __shared__ double sh[NT / 64][NV];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        double o[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) o[q] = q < nv ? __shfl_xor(acc[q], off) : 0.0;
#pragma unroll
        for (int q = 0; q < NV; ++q) acc[q] = q < nsum ? acc[q] + o[q] : fmin(acc[q], o[q]);
    }
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q)
            if (q < nv) sh[wave][q] = acc[q];
    }
    __syncthreads();
    if (threadIdx.x < nv) {
        const int q = threadIdx.x;
        double v = sh[0][q];
        for (int w = 1; w < NT / 64; ++w) v = q < nsum ? v + sh[w][q] : fmin(v, sh[w][q]);
        part[(int64_t)blockIdx.x * nv + q] = v;
    }
}

// The last kernel before each host wait publishes its results: every wave waits until its
// own stores are acknowledged, and after the barrier thread 0 writes them back to system
// scope, then writes the call's sequence number to the flag in the mapped host buffer, on
// which the host spins instead of waiting for the stream to drain.  One workgroup only; flag
// null publishes nothing.
__device__ __forceinline__ void publish(uint64_t *flag, uint64_t seq) {
    if (!flag) return; // (uniform)
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence_system();
        *reinterpret_cast<volatile uint64_t *>(flag) = seq;
        __threadfence_system();
    }
}

// The rows are cut into FIN_CH consecutive chunks; thread (q, c) combines quantity q over
// the rows of chunk c in block order, then out[q] combines the chunk results in chunk order.
// The order is fixed (results do not depend on timing).  A chunk's rows are requested
// FIN_U at a time with no load behind a branch (rows past the chunk read row 0 and are
// dropped), and 1,024 threads take every (quantity, chunk) pair of the solver's largest
// reductions in one to four rounds.
constexpr int FIN_CH = 16;
constexpr int FIN_NT = 1024;
constexpr int FIN_U = 16;
constexpr int FIN_NV = MAXNV > MAXD * (MAXD + 1) / 2 ? MAXNV : MAXD * (MAXD + 1) / 2;

// Also copies ncopy doubles from copy_src to copy_dst (the objective's terms, taken along to the
// host buffer by the same launch).
__global__ __launch_bounds__(FIN_NT) void k_finish(const double *__restrict__ part, int nblk, int nv, int nsum,
                                                   double *__restrict__ out, const double *__restrict__ copy_src,
                                                   int ncopy, double *__restrict__ copy_dst, uint64_t *flag,
                                                   uint64_t seq) {
    if (threadIdx.x < ncopy) copy_dst[threadIdx.x] = copy_src[threadIdx.x];
    __shared__ double sh[FIN_CH][FIN_NV];
    const int per = (nblk + FIN_CH - 1) / FIN_CH;
    for (int e = threadIdx.x; e < nv * FIN_CH; e += FIN_NT) {
        const int q = e % nv, c = e / nv;
        const int b0 = c * per, b1 = min(nblk, b0 + per);
        const bool add = q < nsum;
        double v = add ? 0.0 : INF;
        for (int u0 = b0; u0 < b1; u0 += FIN_U) {
            double pv[FIN_U];
#pragma unroll
            for (int u = 0; u < FIN_U; ++u) {
                const int b = u0 + u;
                pv[u] = part[(int64_t)(b < b1 ? b : 0) * nv + q];
            }
#pragma unroll
            for (int u = 0; u < FIN_U; ++u)
                if (u0 + u < b1) v = add ? v + pv[u] : fmin(v, pv[u]);
        }
        sh[c][q] = v;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < nv; q += FIN_NT) {
        double v = sh[0][q];
        for (int c = 1; c < FIN_CH; ++c) v = q < nsum ? v + sh[c][q] : fmin(v, sh[c][q]);
        out[q] = v;
    }
    publish(flag, seq);
}

// The stored pairs at element i: ys[j] = Y_j[i], ss[j] = S_j[i] for j < k, zero after.
// Unused slots read slot 0 (always allocated) and are masked by a select, so no load sits
// behind a branch or next to its use: all 2 MAXM loads of a thread are in flight together
// instead of one memory latency per stored pair.
__device__ __forceinline__ void load_pairs(const double *__restrict__ S, const double *__restrict__ Y, int64_t n,
                                           const Slots &sl, int64_t i, double (&ys)[MAXM], double (&ss)[MAXM]) {
#pragma unroll
    for (int j = 0; j < MAXM; ++j) {
        const bool on = j < sl.k;
        const int64_t o = (int64_t)(on ? sl.idx[j] : 0) * n + i;
        const double yv = Y[o], sv = S[o];
        ys[j] = on ? yv : 0.0;
        ss[j] = on ? sv : 0.0;
    }
}

// w_i . u with w_i = (Y_0[i] .. Y_{k-1}[i], theta S_0[i] .. theta S_{k-1}[i]),
// u = (uy, us) (entries of u past the stored pairs are zero)
__device__ __forceinline__ double wdot(const double (&ys)[MAXM], const double (&ss)[MAXM], double theta,
                                       const Half &uy, const Half &us) {
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int j = 0; j < MAXM; ++j) {
        a += ys[j] * uy.v[j];
        b += ss[j] * us.v[j];
    }
    return a + theta * b;
}

// ---------------------------------------------------------------- elementwise steps
__global__ __launch_bounds__(NT) void k_start(const ivx_real *__restrict__ xin, int64_t n, int pos,
                                              double *__restrict__ x, ivx_real *__restrict__ sky) {
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        double v = (double)xin[i];
        if (pos && !(v > 0.0)) v = 0.0;
        x[i] = v;
        sky[i] = (ivx_real)v;
    }
}

__global__ __launch_bounds__(NT) void k_out(const double *__restrict__ x, int64_t n, ivx_real *__restrict__ xo) {
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) xo[i] = (ivx_real)x[i];
}

__global__ __launch_bounds__(NT) void k_trial(const double *__restrict__ x, const double *__restrict__ d,
                                              const double *__restrict__ xbar, double stp, int use_bar, int64_t n,
                                              double *__restrict__ xt, ivx_real *__restrict__ sky) {
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        const double v = use_bar ? xbar[i] : x[i] + stp * d[i];
        xt[i] = v;
        sky[i] = (ivx_real)v;
    }
}

// g = grad (FP64); sums: [g.d]; minima: [-|P(x - g) - x|]
__global__ __launch_bounds__(NT) void k_take_grad(const ivx_real *__restrict__ grad, const double *__restrict__ x,
                                                  const double *__restrict__ d, int64_t n, int pos,
                                                  double *__restrict__ g, double *__restrict__ part) {
    double acc[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        const double gi = (double)grad[i];
        g[i] = gi;
        if (d) acc[0] += gi * d[i];
        const double xi = x[i];
        const double pr = pos ? fmax(xi - gi, 0.0) - xi : -gi;
        acc[1] = fmin(acc[1], -fabs(pr));
    }
    block_reduce<2>(acc, 2, 1, part);
}

// Cauchy set-up: breakpoints, steepest-descent direction with fixed variables removed.
// sums: [d.d, #finite breakpoints, #fixed at start, Y_j.d (MAXM), S_j.d (MAXM)]; minima: [t_min]
__global__ __launch_bounds__(NT) void k_cp_init(const double *__restrict__ x, const double *__restrict__ g, int64_t n,
                                                int pos, const double *__restrict__ S, const double *__restrict__ Y,
                                                Slots sl, double *__restrict__ t, double *__restrict__ d,
                                                double *__restrict__ key, int *__restrict__ val,
                                                uint8_t *__restrict__ fixed, double *__restrict__ part,
                                                const double *__restrict__ msrc, int nm, double *__restrict__ mdst) {
    // block 0 also moves the host's M (mapped memory) to the device copy the walk reads
    if (blockIdx.x == 0)
        for (int e = threadIdx.x; e < nm; e += NT) mdst[e] = msrc[e];
    double acc[MAXNV];
#pragma unroll
    for (int q = 0; q < MAXNV; ++q) acc[q] = 0.0;
    double tmin = INF;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        const double gi = g[i];
        const double ti = (pos && gi > 0.0) ? x[i] / gi : INF;
        const bool fx = ti == 0.0;
        const double di = fx ? 0.0 : -gi;
        const bool br = ti > 0.0 && ti < INF;
        t[i] = ti;
        d[i] = di;
        key[i] = br ? ti : INF;
        val[i] = (int)i;
        fixed[i] = fx ? 1 : 0;
        acc[0] += di * di;
        acc[1] += br ? 1.0 : 0.0;
        acc[2] += fx ? 1.0 : 0.0;
        double ys[MAXM], ss[MAXM];
        load_pairs(S, Y, n, sl, i, ys, ss);
#pragma unroll
        for (int j = 0; j < MAXM; ++j) {
            acc[3 + j] += ys[j] * di;
            acc[3 + MAXM + j] += ss[j] * di;
        }
        if (br) tmin = fmin(tmin, ti);
    }
    acc[CP_NS] = tmin;
    block_reduce<MAXNV>(acc, CP_NS + 1, CP_NS, part);
}

// per sorted breakpoint j (and the closing element j = K): q_j, dt_j, g_j, z_j
__global__ __launch_bounds__(NT) void k_cp_q(const double *__restrict__ skey, const int *__restrict__ sidx, int64_t K,
                                             const double *__restrict__ x, const double *__restrict__ g,
                                             const double *__restrict__ S, const double *__restrict__ Y, int64_t n,
                                             Slots sl, double theta, double *__restrict__ Q, double *__restrict__ DT,
                                             double *__restrict__ GB, double *__restrict__ ZB) {
    const int64_t K1 = K + 1;
    const int D = 2 * sl.k;
    for (int64_t j = (int64_t)blockIdx.x * NT + threadIdx.x; j < K1; j += (int64_t)gridDim.x * NT) {
        if (j < K) {
            const int64_t b = sidx[j];
            const double gb = g[b];
            double ys[MAXM], ss[MAXM];
            load_pairs(S, Y, n, sl, b, ys, ss);
#pragma unroll
            for (int c = 0; c < MAXM; ++c) {
                if (c < sl.k) {
                    Q[(int64_t)c * K1 + j] = gb * ys[c];
                    Q[(int64_t)(sl.k + c) * K1 + j] = gb * theta * ss[c];
                }
            }
            DT[j] = skey[j] - (j > 0 ? skey[j - 1] : 0.0);
            GB[j] = gb;
            ZB[j] = -x[b];
        } else {
            for (int c = 0; c < D; ++c) Q[(int64_t)c * K1 + j] = 0.0;
            DT[j] = INF;
            GB[j] = 0.0;
            ZB[j] = 0.0;
        }
    }
}

// ------------------------------------------------------------------ scans
// Exclusive prefix sums along each row of a [rows][L] array, three passes, fixed order.
__device__ __forceinline__ double block_exscan(double v, double &total) {
    __shared__ double sh[NT / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double inc = v;
    for (int off = 1; off < 64; off <<= 1) {
        const double o = __shfl_up(inc, off);
        if (lane >= off) inc += o;
    }
    if (lane == 63) sh[wave] = inc;
    __syncthreads();
    double base = 0.0;
    total = 0.0;
    for (int w = 0; w < NT / 64; ++w) {
        if (w < wave) base += sh[w];
        total += sh[w];
    }
    __syncthreads();
    return base + inc - v;
}

__global__ __launch_bounds__(NT) void k_scan_sums(const double *__restrict__ in, int64_t L, int nb,
                                                  double *__restrict__ bsum) {
    const int row = blockIdx.y;
    const int64_t base = (int64_t)blockIdx.x * SEG;
    double s = 0.0;
    for (int e = 0; e < 4; ++e) {
        const int64_t j = base + (int64_t)threadIdx.x * 4 + e;
        if (j < L) s += in[(int64_t)row * L + j];
    }
    double tot;
    (void)block_exscan(s, tot);
    if (threadIdx.x == 0) bsum[(int64_t)row * nb + blockIdx.x] = tot;
}

__global__ __launch_bounds__(NT) void k_scan_bsums(double *__restrict__ bsum, int nb) {
    const int row = blockIdx.x;
    double carry = 0.0;
    for (int b0 = 0; b0 < nb; b0 += NT) {
        const int b = b0 + threadIdx.x;
        const double v = b < nb ? bsum[(int64_t)row * nb + b] : 0.0;
        double tot;
        const double ex = block_exscan(v, tot);
        if (b < nb) bsum[(int64_t)row * nb + b] = carry + ex;
        carry += tot;
    }
}

__global__ __launch_bounds__(NT) void k_scan_apply(const double *__restrict__ in, int64_t L, int nb,
                                                   const double *__restrict__ bsum, double *__restrict__ out) {
    const int row = blockIdx.y;
    const int64_t base = (int64_t)blockIdx.x * SEG + (int64_t)threadIdx.x * 4;
    double v[4], s = 0.0;
    for (int e = 0; e < 4; ++e) {
        const int64_t j = base + e;
        v[e] = j < L ? in[(int64_t)row * L + j] : 0.0;
        s += v[e];
    }
    double tot;
    // bsum null: a single segment, whose carry is 0
    const double carry = bsum ? bsum[(int64_t)row * nb + blockIdx.x] : 0.0;
    double run = carry + block_exscan(s, tot);
    for (int e = 0; e < 4; ++e) {
        const int64_t j = base + e;
        if (j < L) out[(int64_t)row * L + j] = run;
        run += v[e];
    }
}

// k_cp_a and k_cp_e give each breakpoint j a quad of lanes: lane r of the quad takes rows
// a = r, r + 4, ... of M q_j, and the quad adds its four partial sums in a fixed order
// ((l0 + l1) + (l2 + l3), the same bits on every lane).  Four times the waves of one lane
// per breakpoint keep loads in flight while others compute.
constexpr int QL = 4;               // lanes per breakpoint
constexpr int RPL = MAXD / QL;      // rows of M per lane
static_assert(MAXD % QL == 0, "rows must split evenly over the quad");

__device__ __forceinline__ double quad_sum(double v) {
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    return v;
}

// M (zero past D) and p0 into LDS
__device__ __forceinline__ void load_m(const double *__restrict__ Mdev, int D, double *Ms) {
    for (int e = threadIdx.x; e < MAXD * MAXD; e += NT) {
        const int a = e / MAXD, b = e % MAXD;
        Ms[e] = (a < D && b < D) ? Mdev[a * D + b] : 0.0;
    }
}

// Rows a >= D of M are zero in LDS, so the rows past D of q, P and C (read from row 0 of
// their arrays: finite values) contribute exactly nothing and need no mask.  D = 0 (no
// stored pairs) reads no rows at all: the arrays may not hold finite values yet.

// a_j = theta g_j^2 + 2 q_j.M P_j + q_j.M q_j  and  v_j = dt_j P_j  (P_j = p0 + Pex_j)
__global__ __launch_bounds__(NT) void k_cp_a(const double *__restrict__ Q, const double *__restrict__ Pex,
                                             const double *__restrict__ DT, const double *__restrict__ GB, int64_t K1,
                                             int D, const double *__restrict__ Mdev, Vec p0, double theta,
                                             double *__restrict__ A, double *__restrict__ V) {
    __shared__ double Ms[MAXD * MAXD];
    __shared__ double p0s[MAXD];
    load_m(Mdev, D, Ms);
    if (threadIdx.x < MAXD) p0s[threadIdx.x] = threadIdx.x < D ? p0.v[threadIdx.x] : 0.0;
    __syncthreads();
    const int r = threadIdx.x & (QL - 1);
    const int64_t stride = (int64_t)gridDim.x * (NT / QL);
    // the quad shares j, so its lanes enter and leave the loop together
    for (int64_t j = (int64_t)blockIdx.x * (NT / QL) + (threadIdx.x / QL); j < K1; j += stride) {
        const double gb = GB[j], dt = DT[j];
        double qMP = 0.0, qMq = 0.0;
        if (D > 0) {
            double q[MAXD], P[RPL], qa[RPL];
#pragma unroll
            for (int c = 0; c < MAXD; ++c) q[c] = Q[(int64_t)(c < D ? c : 0) * K1 + j];
#pragma unroll
            for (int t = 0; t < RPL; ++t) {
                const int a = r + QL * t;
                const int64_t o = (int64_t)(a < D ? a : 0) * K1 + j;
                P[t] = p0s[a] + Pex[o];
                qa[t] = Q[o]; // this lane's rows of q again (cache hits), not a register pick
            }
#pragma unroll
            for (int t = 0; t < RPL; ++t) {
                const int a = r + QL * t;
                double mq = 0.0;
#pragma unroll
                for (int b = 0; b < MAXD; ++b) mq += Ms[a * MAXD + b] * q[b];
                qMP += mq * P[t];
                qMq += mq * qa[t];
            }
            // every lane stores all its rows: V has MAXD rows, those past D are never read, and a
            // store guarded per lane made the compiler spill this kernel's registers
#pragma unroll
            for (int t = 0; t < RPL; ++t)
                V[(int64_t)(r + QL * t) * K1 + j] = (dt < INF) ? dt * P[t] : 0.0;
        }
        qMP = quad_sum(qMP);
        qMq = quad_sum(qMq);
        if (r == 0) A[j] = theta * gb * gb + 2.0 * qMP + qMq;
    }
}

// e_j = dt_j f''_j + g_j^2 + theta g_j z_j - q_j.M C_{j+1},  C_{j+1} = Cex_j + v_j
__global__ __launch_bounds__(NT) void k_cp_e(const double *__restrict__ Q, const double *__restrict__ Cex,
                                             const double *__restrict__ V, const double *__restrict__ Aex,
                                             const double *__restrict__ DT, const double *__restrict__ GB,
                                             const double *__restrict__ ZB, int64_t K1, int D,
                                             const double *__restrict__ Mdev, double fpp0, double theta,
                                             double *__restrict__ E) {
    __shared__ double Ms[MAXD * MAXD];
    load_m(Mdev, D, Ms);
    __syncthreads();
    const int r = threadIdx.x & (QL - 1);
    const int64_t stride = (int64_t)gridDim.x * (NT / QL);
    for (int64_t j = (int64_t)blockIdx.x * (NT / QL) + (threadIdx.x / QL); j < K1; j += stride) {
        const double dt = DT[j];
        if (!(dt < INF)) { // uniform over the quad
            if (r == 0) E[j] = 0.0;
            continue;
        }
        double qMC = 0.0;
        if (D > 0) {
            double q[MAXD], C[RPL];
#pragma unroll
            for (int c = 0; c < MAXD; ++c) q[c] = Q[(int64_t)(c < D ? c : 0) * K1 + j];
#pragma unroll
            for (int t = 0; t < RPL; ++t) {
                const int a = r + QL * t;
                const int64_t o = (int64_t)(a < D ? a : 0) * K1 + j;
                C[t] = Cex[o] + V[o];
            }
#pragma unroll
            for (int t = 0; t < RPL; ++t) {
                const int a = r + QL * t;
                double mq = 0.0;
#pragma unroll
                for (int b = 0; b < MAXD; ++b) mq += Ms[a * MAXD + b] * q[b];
                qMC += mq * C[t];
            }
        }
        qMC = quad_sum(qMC);
        if (r == 0) {
            const double gb = GB[j];
            const double f2 = fpp0 - Aex[j];
            E[j] = dt * f2 + gb * gb + theta * gb * ZB[j] - qMC;
        }
    }
}

// The breakpoints below a threshold tau, sorted, in one workgroup: exactly a prefix of the full
// stable sort (ascending IEEE bit patterns, ties by variable index), because every breakpoint
// below tau precedes every other one.  tau is the value of rank ~SEL_TARGET / (n / SEL_SAMPLES)
// among SEL_SAMPLES keys at hashed positions (s * 2654435761 mod n: a fixed stride would alias
// with the image rows), so that about SEL_TARGET breakpoints lie below it;
// when all K finite breakpoints fit the LDS list, tau = +inf selects them all and the prefix is
// the whole walk.  The gathered pairs arrive in any order (LDS atomic slots); each then moves
// to its rank, the number of pairs smaller in (key, index) (unique pairs: a permutation, and no
// dependence on the arrival order).  A pair's count is split over
// SEL_NT / c threads, each over its own run of the list, and the parts are summed with integer
// LDS adds (exact in any order).  out[0] = the prefix length, or -1 when more than SEL_CAP
// breakpoints lie below tau.
constexpr int SEL_NT = 1024;
constexpr int SEL_CAP = 1024;
constexpr int SEL_SAMPLES = 512;
constexpr int SEL_TARGET = 192;
constexpr uint64_t KEY_INF = 0x7FF0000000000000ull; // +inf, the key of a variable without breakpoint
// One workgroup reads every key: beyond this many variables the full sort's launches over the
// whole chip cost less than that single read, and the search sorts everything at once.
constexpr int64_t SEL_MAX_N = int64_t(1) << 24;
static_assert(SEL_CAP <= SEL_NT, "one thread per gathered pair");

__global__ __launch_bounds__(SEL_NT) void k_cp_select(const uint64_t *__restrict__ key, int64_t n, int64_t K,
                                                      uint64_t *__restrict__ skey, uint32_t *__restrict__ sidx,
                                                      double *__restrict__ out, uint64_t *flag, uint64_t seq) {
    __shared__ uint64_t kb[SEL_CAP];
    __shared__ uint32_t ib[SEL_CAP];
    __shared__ int rk[SEL_CAP];
    __shared__ int cnt;
    __shared__ unsigned long long tau;
    const int tid = threadIdx.x;
    if (tid == 0) {
        tau = KEY_INF;
        cnt = 0;
    }
    if (tid < SEL_CAP) rk[tid] = 0;
    if (K > SEL_CAP) {
        // the sample of rank r (0-based, ties by position): r + 1 rounds of a block minimum over
        // the samples not taken yet (r is 1 for n = 65,536; counting every sample's rank reads
        // ns^2 keys through LDS and was slower)
        const int64_t ns = n < SEL_SAMPLES ? n : SEL_SAMPLES;
        const int64_t stride = n / ns;
        int64_t r = SEL_TARGET / stride;
        r = r < 1 ? 1 : (r > ns - 1 ? ns - 1 : r);
        uint64_t v = ~0ull;
        if (tid < ns) v = key[(int64_t)(((uint64_t)tid * 2654435761ull) % (uint64_t)n)];
        __shared__ uint64_t wmin[SEL_NT / 64];
        __shared__ int wpos[SEL_NT / 64];
        const int lane = tid & 63, wave = tid >> 6;
        uint64_t last = ~0ull;
        for (int64_t round = 0; round <= r; ++round) {
            uint64_t m = v;
            int pm = tid;
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) {
                const uint64_t mo = __shfl_xor(m, o);
                const int po = __shfl_xor(pm, o);
                if (mo < m || (mo == m && po < pm)) {
                    m = mo;
                    pm = po;
                }
            }
            if (lane == 0) {
                wmin[wave] = m;
                wpos[wave] = pm;
            }
            __syncthreads();
            m = wmin[0];
            pm = wpos[0];
            for (int w = 1; w < SEL_NT / 64; ++w)
                if (wmin[w] < m || (wmin[w] == m && wpos[w] < pm)) {
                    m = wmin[w];
                    pm = wpos[w];
                }
            last = m;
            if (tid == pm) v = ~0ull; // taken
            __syncthreads();
        }
        if (tid == 0) tau = last < KEY_INF ? last : KEY_INF;
    }
    __syncthreads(); // tau is set
    const uint64_t t = tau;
    // SEL_LOADS keys per thread requested together, then kept or passed over.  Positions past
    // the end read the last key and are masked by a select: a load behind a branch would wait
    // for its own round trip before the next one is issued.
    constexpr int SEL_LOADS = 16;
    for (int64_t i0 = 0; i0 < n; i0 += (int64_t)SEL_NT * SEL_LOADS) {
        uint64_t kk[SEL_LOADS];
#pragma unroll
        for (int u = 0; u < SEL_LOADS; ++u) {
            const int64_t i = i0 + (int64_t)u * SEL_NT + tid;
            const uint64_t kv = key[i < n ? i : n - 1];
            kk[u] = i < n ? kv : ~0ull;
        }
#pragma unroll
        for (int u = 0; u < SEL_LOADS; ++u) {
            if (kk[u] < t) {
                const int p = atomicAdd(&cnt, 1);
                if (p < SEL_CAP) {
                    kb[p] = kk[u];
                    ib[p] = (uint32_t)(i0 + (int64_t)u * SEL_NT + tid);
                }
            }
        }
    }
    __syncthreads();
    const int c = cnt;
    if (c > SEL_CAP) { // (uniform) too many below the threshold: the caller sorts them all
        if (tid == 0) out[0] = -1.0;
        publish(flag, seq);
        return;
    }
    if (c > 0) {
        const int P = SEL_NT / c; // >= 1 since c <= SEL_CAP <= SEL_NT
        if (tid < P * c) {
            const int q = tid % c, part = tid / c;
            const int z0 = (int)((int64_t)c * part / P), z1 = (int)((int64_t)c * (part + 1) / P);
            const uint64_t v = kb[q];
            const uint32_t w = ib[q];
            int below = 0;
#pragma unroll 8
            for (int z = z0; z < z1; ++z) {
                const uint64_t u = kb[z];
                const uint32_t iz = ib[z];
                below += (int)(u < v) | ((int)(u == v) & (int)(iz < w));
            }
            atomicAdd(&rk[q], below);
        }
        __syncthreads();
        if (tid < c) {
            const int rank = rk[tid];
            skey[rank] = kb[tid];
            sidx[rank] = ib[tid];
        }
    }
    if (tid == 0) out[0] = (double)c;
    publish(flag, seq);
}

// first j whose segment holds the minimiser (j = K1 - 1 always qualifies)
__global__ __launch_bounds__(NT) void k_cp_find(const double *__restrict__ Eex, const double *__restrict__ Aex,
                                                const double *__restrict__ DT, int64_t K1, double fp0, double fpp0,
                                                int *__restrict__ Jout) {
    for (int64_t j = (int64_t)blockIdx.x * NT + threadIdx.x; j < K1; j += (int64_t)gridDim.x * NT) {
        const double f1 = fp0 + Eex[j];
        const double f2 = fmax(fpp0 - Aex[j], EPS * fpp0);
        const bool stop = (j == K1 - 1) || (-f1 / f2 < DT[j]);
        if (stop) atomicMin(Jout, (int)j);
    }
}

// state at J into out: [P_J (D), Cex_J (D), f'_J, f''_J, t_{J-1}]
__global__ void k_cp_gather(const int *__restrict__ Jin, const double *__restrict__ Pex,
                            const double *__restrict__ Cex, const double *__restrict__ Eex,
                            const double *__restrict__ Aex, const double *__restrict__ skey, int64_t K1, int D,
                            Vec p0, double fp0, double fpp0, double *__restrict__ out, uint64_t *flag, uint64_t seq) {
    const int J = *Jin;
    const int c = threadIdx.x;
    if (c < D) {
        out[c] = p0.v[c] + Pex[(int64_t)c * K1 + J];
        out[D + c] = Cex[(int64_t)c * K1 + J];
    }
    if (c == 0) {
        out[2 * D] = fp0 + Eex[J];
        out[2 * D + 1] = fpp0 - Aex[J];
        out[2 * D + 2] = J > 0 ? skey[J - 1] : 0.0;
        out[2 * D + 3] = (double)J;
    }
    publish(flag, seq);
}

__global__ void k_set_int(int *__restrict__ p, int v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

__global__ __launch_bounds__(NT) void k_cp_fix(const int *__restrict__ Jin, const int *__restrict__ sidx,
                                               uint8_t *__restrict__ fixed) {
    const int J = *Jin;
    for (int j = blockIdx.x * NT + threadIdx.x; j < J; j += gridDim.x * NT) fixed[sidx[j]] = 1;
}

__global__ __launch_bounds__(NT) void k_cp_xc(const double *__restrict__ x, const double *__restrict__ d,
                                              const uint8_t *__restrict__ fixed, double tc, int64_t n,
                                              double *__restrict__ xc) {
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
        xc[i] = fixed[i] ? 0.0 : x[i] + tc * d[i];
}

// ------------------------------------------------------------ subspace step
// r = g + theta (xc - x) - W M c on the free variables; sums: [Y_j.r (MAXM), S_j.r (MAXM)]
__global__ __launch_bounds__(NT) void k_ss_r(const double *__restrict__ x, const double *__restrict__ xc,
                                             const double *__restrict__ g, const uint8_t *__restrict__ fixed,
                                             const double *__restrict__ S, const double *__restrict__ Y, int64_t n,
                                             Slots sl, double theta, Half mcy, Half mcs, double *__restrict__ r,
                                             double *__restrict__ part) {
    double acc[MAXD];
#pragma unroll
    for (int q = 0; q < MAXD; ++q) acc[q] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        double ys[MAXM], ss[MAXM];
        load_pairs(S, Y, n, sl, i, ys, ss);
        double ri = 0.0;
        if (!fixed[i]) ri = g[i] + theta * (xc[i] - x[i]) - wdot(ys, ss, theta, mcy, mcs);
        r[i] = ri;
#pragma unroll
        for (int j = 0; j < MAXM; ++j) {
            acc[j] += ys[j] * ri;
            acc[MAXM + j] += ss[j] * ri;
        }
    }
    block_reduce<MAXD>(acc, MAXD, MAXD, part);
}

// Gram matrix of (Y_0..Y_{k-1}, S_0..S_{k-1}) over the free rows, upper triangle row-major;
// every thread owns whole entries, so no block reduction is needed.
constexpr int GCH = 64;
__global__ __launch_bounds__(NT) void k_ss_gram(const uint8_t *__restrict__ fixed, const double *__restrict__ S,
                                                const double *__restrict__ Y, int64_t n, Slots sl,
                                                double *__restrict__ part) {
    __shared__ double sh[GCH][MAXD + 1];
    __shared__ int slot[MAXM];
    const int k = sl.k, D = 2 * k, np = D * (D + 1) / 2;
    if (threadIdx.x < MAXM) slot[threadIdx.x] = threadIdx.x < k ? sl.idx[threadIdx.x] : 0;
    constexpr int PPT = (MAXD * (MAXD + 1) / 2 + NT - 1) / NT;
    double acc[PPT];
    int pa[PPT], pb[PPT];
#pragma unroll
    for (int e = 0; e < PPT; ++e) {
        acc[e] = 0.0;
        int p = threadIdx.x + e * NT, a = 0;
        if (p >= np) p = 0;
        while (p >= D - a) {
            p -= D - a;
            ++a;
        }
        pa[e] = a;
        pb[e] = a + p;
    }
    __syncthreads(); // slot[] is read by every thread below
    for (int64_t r0 = (int64_t)blockIdx.x * GCH; r0 < n; r0 += (int64_t)gridDim.x * GCH) {
        // stage 64 rows x D columns: all of a thread's loads first (out-of-range entries read
        // row 0 and are masked), then the LDS stores.  A thread's row is the same at every
        // step (NT is a multiple of GCH), so its flag byte is read once.
        constexpr int GIT = GCH * MAXD / NT;
        static_assert(NT % GCH == 0, "one row per thread across the staging steps");
        const int64_t i = r0 + threadIdx.x % GCH;
        const int64_t ic = i < n ? i : 0;
        const uint8_t fx = fixed[ic];
        double v[GIT];
#pragma unroll
        for (int it = 0; it < GIT; ++it) {
            const int c = (threadIdx.x + it * NT) / GCH;
            const int sj = c < k ? slot[c] : slot[min(c - k, MAXM - 1)];
            v[it] = (c < k ? Y : S)[(int64_t)sj * n + ic];
        }
        const bool live = i < n && !fx;
#pragma unroll
        for (int it = 0; it < GIT; ++it) {
            const int c = (threadIdx.x + it * NT) / GCH;
            v[it] = (live && c < D) ? v[it] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < GIT; ++it) {
            const int e = threadIdx.x + it * NT;
            sh[e % GCH][e / GCH] = v[it];
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < PPT; ++e) {
            if (threadIdx.x + e * NT >= np) continue;
            double s = 0.0;
#pragma unroll 4
            for (int rr = 0; rr < GCH; ++rr) s += sh[rr][pa[e]] * sh[rr][pb[e]];
            acc[e] += s;
        }
    }
#pragma unroll
    for (int e = 0; e < PPT; ++e) {
        const int p = threadIdx.x + e * NT;
        if (p < np) part[(int64_t)blockIdx.x * np + p] = acc[e];
    }
}

// du = -r/theta - (w.u)/theta^2; xbar = P(xc + du) on the free variables
// sums: [(xbar - x).g]; minima: [min over du<0 of -xc/du]
__global__ __launch_bounds__(NT) void k_ss_du(const double *__restrict__ x, const double *__restrict__ xc,
                                              const double *__restrict__ g, const double *__restrict__ r,
                                              const uint8_t *__restrict__ fixed, const double *__restrict__ S,
                                              const double *__restrict__ Y, int64_t n, Slots sl, double theta,
                                              Half uy, Half us, int pos, double *__restrict__ du, double *__restrict__ xbar,
                                              double *__restrict__ part) {
    double acc[2] = {0.0, INF};
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        // every load ahead of the branch (r holds 0 on the fixed rows), so none waits alone
        const double xci = xc[i], ri = r[i], xi = x[i], gi = g[i];
        const uint8_t fx = fixed[i];
        double ys[MAXM], ss[MAXM];
        load_pairs(S, Y, n, sl, i, ys, ss);
        double dui = 0.0, xb = xci;
        if (!fx) {
            dui = -ri / theta - wdot(ys, ss, theta, uy, us) / (theta * theta);
            xb = xci + dui;
            if (pos) {
                xb = fmax(xb, 0.0);
                if (dui < 0.0) acc[1] = fmin(acc[1], -xci / dui);
            }
        }
        du[i] = dui;
        xbar[i] = xb;
        acc[0] += (xb - xi) * gi;
    }
    block_reduce<2>(acc, 2, 1, part);
}

__global__ __launch_bounds__(NT) void k_ss_trunc(const double *__restrict__ xc, const double *__restrict__ du,
                                                 const uint8_t *__restrict__ fixed, double alpha, int64_t n,
                                                 double *__restrict__ xbar) {
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
        xbar[i] = fixed[i] ? xc[i] : xc[i] + alpha * du[i];
}

// d = xbar - x; sums: [d.d, g.d]; minima: [min over d<0 of -x/d]
__global__ __launch_bounds__(NT) void k_dir(const double *__restrict__ x, const double *__restrict__ xbar,
                                            const double *__restrict__ g, int64_t n, int pos, double *__restrict__ d,
                                            double *__restrict__ part) {
    double acc[3] = {0.0, 0.0, INF};
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        const double di = xbar[i] - x[i];
        d[i] = di;
        acc[0] += di * di;
        acc[1] += g[i] * di;
        if (pos && di < 0.0) acc[2] = fmin(acc[2], -x[i] / di);
    }
    block_reduce<3>(acc, 3, 2, part);
}

// accepted step: s = xt - x, y = gt - g into the spare slot;
// sums: [s.y, y.y, g.s, s.s, s.Y_j, S_j.y, s.S_j (MAXM each)]; minima: [-pg(xt)]
__global__ __launch_bounds__(NT) void k_update(const double *__restrict__ x, const double *__restrict__ xt,
                                               const double *__restrict__ g, const double *__restrict__ gt, int64_t n,
                                               int pos, double *__restrict__ S, double *__restrict__ Y, int spare,
                                               Slots sl, double *__restrict__ part) {
    double acc[MAXNV];
#pragma unroll
    for (int q = 0; q < MAXNV; ++q) acc[q] = 0.0;
    double mn = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        // the stored pairs never include the spare slot; an unused slot may alias it, but
        // only this thread touches element i and the masked value is discarded
        double ys[MAXM], ss[MAXM];
        load_pairs(S, Y, n, sl, i, ys, ss);
        const double s = xt[i] - x[i], y = gt[i] - g[i];
        S[(int64_t)spare * n + i] = s;
        Y[(int64_t)spare * n + i] = y;
        acc[0] += s * y;
        acc[1] += y * y;
        acc[2] += g[i] * s;
        acc[3] += s * s;
#pragma unroll
        for (int j = 0; j < MAXM; ++j) {
            acc[4 + j] += s * ys[j];
            acc[4 + MAXM + j] += ss[j] * y;
            acc[4 + 2 * MAXM + j] += s * ss[j];
        }
        const double xi = xt[i], gi = gt[i];
        const double pr = pos ? fmax(xi - gi, 0.0) - xi : -gi;
        mn = fmin(mn, -fabs(pr));
    }
    acc[UP_NS] = mn;
    block_reduce<MAXNV>(acc, UP_NS + 1, UP_NS, part);
}

// ------------------------------------------------------------ host linear algebra
// Solve A X = B (A n x n, B n x r, row-major) by Gaussian elimination with partial
// pivoting; returns false if A is singular.
bool solve_dense(std::vector<double> A, std::vector<double> &B, int n, int r) {
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int i = c + 1; i < n; ++i)
            if (std::fabs(A[i * n + c]) > std::fabs(A[piv * n + c])) piv = i;
        if (!(std::fabs(A[piv * n + c]) > 0.0)) return false;
        if (piv != c) {
            for (int j = 0; j < n; ++j) std::swap(A[c * n + j], A[piv * n + j]);
            for (int j = 0; j < r; ++j) std::swap(B[c * r + j], B[piv * r + j]);
        }
        for (int i = c + 1; i < n; ++i) {
            const double f = A[i * n + c] / A[c * n + c];
            if (f == 0.0) continue;
            for (int j = c; j < n; ++j) A[i * n + j] -= f * A[c * n + j];
            for (int j = 0; j < r; ++j) B[i * r + j] -= f * B[c * r + j];
        }
    }
    for (int c = n - 1; c >= 0; --c) {
        for (int j = 0; j < r; ++j) {
            double s = B[c * r + j];
            for (int i = c + 1; i < n; ++i) s -= A[c * n + i] * B[i * r + j];
            B[c * r + j] = s / A[c * n + c];
        }
    }
    return true;
}

// ------------------------------------------------------------ line search (host)
// Strong-Wolfe search of More & Thuente (1994): an interval of uncertainty [stx, sty]
// updated by the four-case safeguarded cubic/quadratic step, with the modified function
// psi(a) = f(a) - f(0) - ftol a f'(0) while no point of sufficient decrease and
// non-negative slope has been seen.
struct WolfeSearch {
    double ftol = 1e-3, gtol = 0.9, xtol = 0.1, stpmin = 0.0, stpmax = 1e10;
    bool brackt = false;
    int stage = 1;
    double finit = 0, ginit = 0, gtest = 0, width = 0, width1 = 0;
    double stx = 0, fx = 0, gx = 0, sty = 0, fy = 0, gy = 0, stmin = 0, stmax = 0, stp = 0;

    void start(double f0, double g0, double stp0) {
        brackt = false;
        stage = 1;
        finit = f0;
        ginit = g0;
        gtest = ftol * g0;
        width = stpmax - stpmin;
        width1 = 2.0 * width;
        stx = sty = 0.0;
        fx = fy = f0;
        gx = gy = g0;
        stmin = 0.0;
        stmax = stp0 + 4.0 * stp0;
        stp = stp0;
    }

    // 0: evaluate at stp again, 1: converged, 2: stopped with a warning (accept stp)
    int next(double f, double g) {
        const double ftest = finit + stp * gtest;
        if (stage == 1 && f <= ftest && g >= 0.0) stage = 2;
        if (brackt && (stp <= stmin || stp >= stmax)) return 2;
        if (brackt && stmax - stmin <= xtol * stmax) return 2;
        if (stp == stpmax && f <= ftest && g <= gtest) return 2;
        if (stp == stpmin && (f > ftest || g >= gtest)) return 2;
        if (f <= ftest && std::fabs(g) <= gtol * (-ginit)) return 1;
        double nstp;
        if (stage == 1 && f <= fx && f > ftest) {
            double fxm = fx - stx * gtest, gxm = gx - gtest, fym = fy - sty * gtest, gym = gy - gtest;
            nstp = safeguarded_step(stx, fxm, gxm, sty, fym, gym, stp, f - stp * gtest, g - gtest);
            fx = fxm + stx * gtest;
            fy = fym + sty * gtest;
            gx = gxm + gtest;
            gy = gym + gtest;
        } else {
            nstp = safeguarded_step(stx, fx, gx, sty, fy, gy, stp, f, g);
        }
        if (brackt) {
            if (std::fabs(sty - stx) >= 0.66 * width1) nstp = stx + 0.5 * (sty - stx);
            width1 = width;
            width = std::fabs(sty - stx);
            stmin = std::min(stx, sty);
            stmax = std::max(stx, sty);
        } else {
            stmin = nstp + 1.1 * (nstp - stx);
            stmax = nstp + 4.0 * (nstp - stx);
        }
        nstp = std::min(std::max(nstp, stpmin), stpmax);
        if ((brackt && (nstp <= stmin || nstp >= stmax)) || (brackt && stmax - stmin <= xtol * stmax)) nstp = stx;
        stp = nstp;
        return 0;
    }

    // Updates the interval end points in place and returns the next trial step.
    double safeguarded_step(double &sx, double &fsx, double &dsx, double &sy, double &fsy, double &dsy, double sp,
                            double fp, double dp) {
        const double lo = stmin, hi = stmax;
        const double sgnd = dp * (dsx / std::fabs(dsx));
        double sf;
        auto cubic_terms = [](double a, double fa, double da, double b, double fb, double db, double &th, double &s) {
            th = 3.0 * (fa - fb) / (b - a) + da + db;
            s = std::max(std::fabs(th), std::max(std::fabs(da), std::fabs(db)));
            return (th / s) * (th / s) - (da / s) * (db / s);
        };
        if (fp > fsx) {
            double th, s;
            const double disc = cubic_terms(sx, fsx, dsx, sp, fp, dp, th, s);
            double gam = s * std::sqrt(disc);
            if (sp < sx) gam = -gam;
            const double p = (gam - dsx) + th, q = ((gam - dsx) + gam) + dp;
            const double sc = sx + (p / q) * (sp - sx);
            const double sq = sx + ((dsx / ((fsx - fp) / (sp - sx) + dsx)) / 2.0) * (sp - sx);
            sf = std::fabs(sc - sx) < std::fabs(sq - sx) ? sc : sc + (sq - sc) / 2.0;
            brackt = true;
        } else if (sgnd < 0.0) {
            double th, s;
            const double disc = cubic_terms(sx, fsx, dsx, sp, fp, dp, th, s);
            double gam = s * std::sqrt(disc);
            if (sp > sx) gam = -gam;
            const double p = (gam - dp) + th, q = ((gam - dp) + gam) + dsx;
            const double sc = sp + (p / q) * (sx - sp);
            const double sq = sp + (dp / (dp - dsx)) * (sx - sp);
            sf = std::fabs(sc - sp) > std::fabs(sq - sp) ? sc : sq;
            brackt = true;
        } else if (std::fabs(dp) < std::fabs(dsx)) {
            double th, s;
            const double disc = cubic_terms(sx, fsx, dsx, sp, fp, dp, th, s);
            double gam = s * std::sqrt(std::max(0.0, disc));
            if (sp > sx) gam = -gam;
            const double p = (gam - dp) + th, q = (gam + (dsx - dp)) + gam;
            const double r = p / q;
            double sc;
            if (r < 0.0 && gam != 0.0) sc = sp + r * (sx - sp);
            else if (sp > sx) sc = hi;
            else sc = lo;
            const double sq = sp + (dp / (dp - dsx)) * (sx - sp);
            if (brackt) {
                sf = std::fabs(sc - sp) < std::fabs(sq - sp) ? sc : sq;
                sf = sp > sx ? std::min(sp + 0.66 * (sy - sp), sf) : std::max(sp + 0.66 * (sy - sp), sf);
            } else {
                sf = std::fabs(sc - sp) > std::fabs(sq - sp) ? sc : sq;
                sf = std::max(std::min(sf, hi), lo);
            }
        } else {
            if (brackt) {
                double th, s;
                const double disc = cubic_terms(sy, fsy, dsy, sp, fp, dp, th, s);
                double gam = s * std::sqrt(disc);
                if (sp > sy) gam = -gam;
                const double p = (gam - dp) + th, q = ((gam - dp) + gam) + dsy;
                sf = sp + (p / q) * (sy - sp);
            } else {
                sf = sp > sx ? hi : lo;
            }
        }
        if (fp > fsx) {
            sy = sp;
            fsy = fp;
            dsy = dp;
        } else {
            if (sgnd < 0.0) {
                sy = sx;
                fsy = fsx;
                dsy = dsx;
            }
            sx = sp;
            fsx = fp;
            dsx = dp;
        }
        return sf;
    }
};

} // namespace

// ================================================================ solver object
struct ivx_lbfgsb {
    ivx_plan *plan = nullptr;
    int64_t n = 0;
    int mmax = 0;
    std::vector<void *> bufs;
    double *x = nullptr, *g = nullptr, *xt = nullptr, *gt = nullptr, *d = nullptr, *xc = nullptr, *xbar = nullptr;
    double *r = nullptr, *du = nullptr, *t = nullptr, *key = nullptr, *key2 = nullptr;
    int *val = nullptr, *val2 = nullptr;
    uint8_t *fixed = nullptr;
    double *S = nullptr, *Y = nullptr;
    double *Q = nullptr, *Pex = nullptr, *V = nullptr, *Cex = nullptr;
    double *DT = nullptr, *GB = nullptr, *ZB = nullptr, *A = nullptr, *Aex = nullptr, *E = nullptr, *Eex = nullptr;
    double *bsum = nullptr;
    double *part = nullptr, *scal = nullptr, *Mdev = nullptr;
    int *Jdev = nullptr;
    ivx_real *sky = nullptr, *grad = nullptr;
    void *sort_tmp = nullptr;
    size_t sort_bytes = 0;
    double *host = nullptr;     // pinned, mapped
    double *host_dev = nullptr; // the same buffer as the device addresses it
    uint64_t seq = 0;           // the last sequence number handed to a publishing kernel
    bool stream_wait = false;   // this solve reads results after the stream drains
};

namespace {

ivx_status lb_alloc(ivx_lbfgsb *s, void **p, size_t bytes) {
    *p = nullptr;
    if (hipMalloc(p, bytes > 0 ? bytes : 1) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(IVX_ENOMEM, "hipMalloc failed in ivx_lbfgsb_create");
    }
    s->bufs.push_back(*p);
    return IVX_OK;
}

template <typename T> ivx_status lb_alloc_t(ivx_lbfgsb *s, T **p, size_t count) {
    void *q = nullptr;
    ivx_status st = lb_alloc(s, &q, count * sizeof(T));
    *p = (T *)q;
    return st;
}

void lb_free(ivx_lbfgsb *s) {
    for (void *p : s->bufs) (void)hipFree(p);
    s->bufs.clear();
    if (s->host) (void)hipHostFree(s->host);
    s->host = nullptr;
}

unsigned grid_of(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(RBLK, (n + NT - 1) / NT)); }

#define LB_HIP(call)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess) return set_error(IVX_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

uint64_t *flag_dev(ivx_lbfgsb *s) { return reinterpret_cast<uint64_t *>(s->host_dev + FLAG); }

// Waits until the kernel handed sequence number seq has published its results.  The host
// spins on the flag in the mapped buffer; past 20 ms (a slow call, or a kernel that failed),
// or at once when the solve asked for stream waits, it waits for the stream, which also
// reports any error.
ivx_status wait_published(ivx_lbfgsb *s, uint64_t seq, hipStream_t st) {
    const volatile uint64_t *f = reinterpret_cast<const volatile uint64_t *>(s->host + FLAG);
    const auto t0 = std::chrono::steady_clock::now();
    for (uint32_t i = 0; !s->stream_wait; ++i) {
        if (*f == seq) {
            std::atomic_thread_fence(std::memory_order_acquire);
            return IVX_OK;
        }
        if ((i & 1023) == 1023 && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(20)) break;
    }
    LB_HIP(hipStreamSynchronize(st));
    if (*f != seq) return set_error(IVX_EHIP, "a solver kernel completed without publishing its result");
    std::atomic_thread_fence(std::memory_order_acquire);
    return IVX_OK;
}

// Sum/min reduce a kernel's block partials into the host buffer at s->host[off..off+nv).
ivx_status reduce_to_host(ivx_lbfgsb *s, unsigned nblk, int nv, int nsum, int off, hipStream_t st) {
    // the finisher writes the few results straight into the mapped host buffer (no copy
    // launch) and publishes them
    const uint64_t q = ++s->seq;
    k_finish<<<1, FIN_NT, 0, st>>>(s->part, (int)nblk, nv, nsum, s->host_dev + off, nullptr, 0, nullptr,
                                   flag_dev(s), q);
    LB_HIP(hipGetLastError());
    return wait_published(s, q, st);
}

ivx_status scan_rows(ivx_lbfgsb *s, const double *in, double *out, int rows, int64_t L, hipStream_t st) {
    const int nb = (int)((L + SEG - 1) / SEG);
    if (nb == 1) {
        // one segment per row (every walk over a sampled prefix): the apply pass alone, with
        // the carry 0 that the two segment passes would have produced
        k_scan_apply<<<dim3(1, rows), NT, 0, st>>>(in, L, 1, nullptr, out);
    } else {
        k_scan_sums<<<dim3(nb, rows), NT, 0, st>>>(in, L, nb, s->bsum);
        k_scan_bsums<<<rows, NT, 0, st>>>(s->bsum, nb);
        k_scan_apply<<<dim3(nb, rows), NT, 0, st>>>(in, L, nb, s->bsum, out);
    }
    LB_HIP(hipGetLastError());
    return IVX_OK;
}

struct Memory {
    int k = 0;
    std::vector<int> order; // slot ids, oldest first
    int spare = 0;
    double theta = 1.0;
    double SY[MAXM][MAXM] = {}, SS[MAXM][MAXM] = {};
    std::vector<double> M; // (2k)^2 row-major

    Slots slots() const {
        Slots sl{};
        for (int j = 0; j < k; ++j) sl.idx[j] = order[j];
        sl.k = k;
        return sl;
    }
    void reset(int mmax) {
        k = 0;
        order.clear();
        spare = 0;
        theta = 1.0;
        M.clear();
        (void)mmax;
    }
    // M = [[-D, L^T], [L, theta S^T S]]^-1
    bool rebuild() {
        const int D = 2 * k;
        M.assign((size_t)D * D, 0.0);
        if (k == 0) return true;
        std::vector<double> K((size_t)D * D, 0.0), I((size_t)D * D, 0.0);
        for (int a = 0; a < k; ++a) {
            K[a * D + a] = -SY[a][a];
            for (int b = 0; b < k; ++b) {
                if (a > b) {
                    K[(k + a) * D + b] = SY[a][b];   // L
                    K[b * D + (k + a)] = SY[a][b];   // L^T
                }
                K[(k + a) * D + (k + b)] = theta * SS[a][b];
            }
        }
        for (int a = 0; a < D; ++a) I[a * D + a] = 1.0;
        if (!solve_dense(K, I, D, D)) return false;
        M = I;
        return true;
    }
};

} // namespace

extern "C" {

ivx_status ivx_lbfgsb_default_options(ivx_lbfgsb_options *o) {
    if (!o) return set_error(IVX_EINVAL, "options pointer is NULL");
    o->m = 10;
    o->maxiter = 15000;
    o->maxfun = 15000;
    o->maxls = 20;
    o->positivity = 1;
    o->full_sort = 0;
    o->stream_wait = 0;
    o->reserved = 0;
    o->ftol = 2.220446049250313e-09;
    o->gtol = 1e-5;
    o->target = -INFINITY;
    return IVX_OK;
}

ivx_status ivx_lbfgsb_create(ivx_plan *plan, int32_t m_max, ivx_lbfgsb **out) {
    if (!out) return set_error(IVX_EINVAL, "out is NULL");
    *out = nullptr;
    if (!plan) return set_error(IVX_EINVAL, "plan is NULL");
    if (m_max < 1 || m_max > MAXM) return set_error(IVX_EINVAL, "m_max must be in [1, 16]");
    const int64_t n = plan_sky_count(plan);
    if (n < 1 || n > (int64_t)INT32_MAX - 2) return set_error(IVX_EINVAL, "plan has no sky or too many pixels");
    ivx_lbfgsb *s = new ivx_lbfgsb();
    s->plan = plan;
    s->n = n;
    s->mmax = m_max;
    const int64_t n1 = n + 1;
    const int D = 2 * m_max;
    const int nb = (int)((n1 + SEG - 1) / SEG);
    ivx_status st = IVX_OK;
    double **vecs[] = {&s->x, &s->g, &s->xt, &s->gt, &s->d, &s->xc, &s->xbar, &s->r, &s->du, &s->t, &s->key, &s->key2};
    for (double **p : vecs)
        if (!st) st = lb_alloc_t(s, p, (size_t)n);
    if (!st) st = lb_alloc_t(s, &s->val, (size_t)n);
    if (!st) st = lb_alloc_t(s, &s->val2, (size_t)n);
    if (!st) st = lb_alloc_t(s, &s->fixed, (size_t)n);
    if (!st) st = lb_alloc_t(s, &s->S, (size_t)(m_max + 1) * n);
    if (!st) st = lb_alloc_t(s, &s->Y, (size_t)(m_max + 1) * n);
    double **rowsv[] = {&s->Q, &s->Pex, &s->Cex};
    for (double **p : rowsv)
        if (!st) st = lb_alloc_t(s, p, (size_t)D * n1);
    if (!st) st = lb_alloc_t(s, &s->V, (size_t)MAXD * n1); // k_cp_a writes MAXD rows
    double **scal1[] = {&s->DT, &s->GB, &s->ZB, &s->A, &s->Aex, &s->E, &s->Eex};
    for (double **p : scal1)
        if (!st) st = lb_alloc_t(s, p, (size_t)n1);
    if (!st) st = lb_alloc_t(s, &s->bsum, (size_t)D * nb + 1);
    // block partials: one reduction's rows, or the Gram matrix's followed by W^T r's (PART_R on)
    if (!st) st = lb_alloc_t(s, &s->part, (size_t)RBLK * (MAXD * (MAXD + 1) / 2 + MAXD));
    if (!st) st = lb_alloc_t(s, &s->scal, SCAL);
    if (!st) st = lb_alloc_t(s, &s->Mdev, (size_t)MAXD * MAXD);
    if (!st) st = lb_alloc_t(s, &s->Jdev, 1);
    if (!st) st = lb_alloc_t(s, &s->sky, (size_t)n);
    if (!st) st = lb_alloc_t(s, &s->grad, (size_t)n);
    if (!st) {
        s->sort_bytes = radix_sort_temp_bytes((int)n, true);
        st = lb_alloc(s, &s->sort_tmp, s->sort_bytes);
    }
    if (!st && hipHostMalloc((void **)&s->host, SCAL * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        s->host = nullptr;
        st = set_error(IVX_ENOMEM, "hipHostMalloc failed in ivx_lbfgsb_create");
    }
    if (!st) std::memset(s->host, 0, SCAL * sizeof(double)); // the flag starts below every sequence number
    if (!st && hipHostGetDevicePointer((void **)&s->host_dev, s->host, 0) != hipSuccess) {
        (void)hipGetLastError();
        st = set_error(IVX_EHIP, "hipHostGetDevicePointer failed in ivx_lbfgsb_create");
    }
    if (st) {
        lb_free(s);
        delete s;
        return st;
    }
    *out = s;
    return IVX_OK;
}

ivx_status ivx_lbfgsb_destroy(ivx_lbfgsb *s) {
    if (!s) return IVX_OK;
    lb_free(s);
    delete s;
    return IVX_OK;
}

ivx_status ivx_lbfgsb_solve(ivx_lbfgsb *s, ivx_real *xio, const ivx_lbfgsb_options *opt_in, double *f_hist,
                            double *t_hist, int64_t hist_cap, ivx_lbfgsb_result *res, void *stream) {
    if (!s || !xio || !res) return set_error(IVX_EINVAL, "solver, x and res are required");
    ivx_lbfgsb_options opt;
    if (opt_in) opt = *opt_in;
    else ivx_lbfgsb_default_options(&opt);
    if (opt.m < 1 || opt.m > s->mmax || opt.maxiter < 0 || opt.maxfun < 1 || opt.maxls < 1 || !(opt.ftol >= 0.0) ||
        !(opt.gtol >= 0.0) || std::isnan(opt.target))
        return set_error(IVX_EINVAL, "bad L-BFGS-B options (m must not exceed the solver's m_max)");
    if (hist_cap < 0 || (hist_cap > 0 && !f_hist)) return set_error(IVX_EINVAL, "bad history buffer");
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = s->n;
    const unsigned G = grid_of(n);
    const int pos = opt.positivity ? 1 : 0;
    const auto t0 = std::chrono::steady_clock::now();
    double *h = s->host;
    s->stream_wait = opt.stream_wait != 0;
    int64_t nfev = 0, nit = 0, nwalk = 0, nwalk_full = 0;
    double f = 0.0, pg = 0.0;
    int reason = IVX_LBFGSB_MAXITER;

    // one objective evaluation at s->sky: gradient into gdst, g.d (if d) and the projected
    // gradient at xcur; returns f
    auto evaluate = [&](const double *xcur, const double *dvec, double *gdst, double &fval, double &gd,
                        double &pgn) -> ivx_status {
        ivx_status e = ivx_objective_grad(s->plan, s->sky, s->grad, s->scal, st);
        if (e != IVX_OK) return e;
        k_take_grad<<<G, NT, 0, st>>>(s->grad, xcur, dvec, n, pos, gdst, s->part);
        // g.d and |pg| and the four terms land in the mapped host buffer: no copy launch
        const uint64_t q = ++s->seq;
        k_finish<<<1, FIN_NT, 0, st>>>(s->part, (int)G, 2, 1, s->host_dev + OFF, s->scal, 4, s->host_dev,
                                       flag_dev(s), q);
        LB_HIP(hipGetLastError());
        if ((e = wait_published(s, q, st)) != IVX_OK) return e;
        fval = h[0];
        gd = h[OFF];
        pgn = -h[OFF + 1];
        if (nfev < hist_cap) {
            f_hist[nfev] = fval;
            if (t_hist) t_hist[nfev] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        }
        ++nfev;
        return IVX_OK;
    };

    ivx_status e;
    k_start<<<G, NT, 0, st>>>(xio, n, pos, s->x, s->sky);
    LB_HIP(hipGetLastError());
    {
        double gd_unused;
        if ((e = evaluate(s->x, nullptr, s->g, f, gd_unused, pg)) != IVX_OK) return e;
    }
    Memory mem;
    const int m = opt.m;
    std::vector<char> used(m + 1, 0);
    auto first_free = [&]() {
        for (int j = 0; j <= m; ++j)
            if (!used[j]) return j;
        return 0;
    };
    mem.reset(m);
    mem.spare = 0;

    if (f <= opt.target) reason = IVX_LBFGSB_TARGET;
    else if (pg <= opt.gtol) reason = IVX_LBFGSB_PGTOL;
    else if (opt.maxiter == 0) reason = IVX_LBFGSB_MAXITER;
    else {
        for (;;) {
            const Slots sl = mem.slots();
            const int k = mem.k, D = 2 * k;
            const double theta = mem.theta;
            // M goes through the mapped host buffer (the stream has drained: no kernel reads it)
            if (k > 0) std::copy(mem.M.begin(), mem.M.begin() + (size_t)D * D, h + MOFF);
            // ---- generalized Cauchy point
            k_cp_init<<<G, NT, 0, st>>>(s->x, s->g, n, pos, s->S, s->Y, sl, s->t, s->d, s->key, s->val, s->fixed,
                                        s->part, s->host_dev + MOFF, k > 0 ? D * D : 0, s->Mdev);
            LB_HIP(hipGetLastError());
            if ((e = reduce_to_host(s, G, CP_NS + 1, CP_NS, OFF, st)) != IVX_OK) return e;
            const double dd = h[OFF], nbr = h[OFF + 1], nfix0 = h[OFF + 2], tmin = h[OFF + CP_NS];
            std::vector<double> p0(D), c(D, 0.0);
            for (int j = 0; j < k; ++j) {
                p0[j] = h[OFF + 3 + j];
                p0[k + j] = theta * h[OFF + 3 + MAXM + j];
            }
            auto quad = [&](const std::vector<double> &a, const std::vector<double> &b) {
                double q = 0.0;
                for (int i = 0; i < D; ++i)
                    for (int j = 0; j < D; ++j) q += a[i] * mem.M[i * D + j] * b[j];
                return q;
            };
            const double fp0 = -dd;
            const double fpp0 = -theta * fp0 - quad(p0, p0);
            double tc = 0.0;
            int64_t nfixed = (int64_t)nfix0;
            if (fp0 < 0.0) {
                const double dtm0 = fpp0 > 0.0 ? -fp0 / fpp0 : 0.0;
                if (nbr < 0.5 || dtm0 < tmin) {
                    tc = std::max(dtm0, 0.0);
                    for (int j = 0; j < D; ++j) c[j] = tc * p0[j];
                } else {
                    const int64_t K = (int64_t)nbr;
                    ++nwalk;
                    Vec p0v{};
                    for (int j = 0; j < D; ++j) p0v.v[j] = p0[j];
                    // the walk over the first Kw sorted breakpoints (key2 / val2), closed by a
                    // last segment to +inf; writes J and the state at its segment
                    int64_t J = 0;
                    double f1 = 0.0, f2 = 0.0, told = 0.0;
                    auto walk = [&](int64_t Kw) -> ivx_status {
                        const int64_t K1 = Kw + 1;
                        const unsigned GK = (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, (K1 + NT - 1) / NT));
                        const unsigned GQ =
                            (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, (QL * K1 + NT - 1) / NT));
                        ivx_status ew;
                        k_cp_q<<<GK, NT, 0, st>>>(s->key2, s->val2, Kw, s->x, s->g, s->S, s->Y, n, sl, theta, s->Q,
                                                  s->DT, s->GB, s->ZB);
                        LB_HIP(hipGetLastError());
                        if (D > 0 && (ew = scan_rows(s, s->Q, s->Pex, D, K1, st)) != IVX_OK) return ew;
                        k_cp_a<<<GQ, NT, 0, st>>>(s->Q, s->Pex, s->DT, s->GB, K1, D, s->Mdev, p0v, theta, s->A, s->V);
                        LB_HIP(hipGetLastError());
                        if ((ew = scan_rows(s, s->A, s->Aex, 1, K1, st)) != IVX_OK) return ew;
                        if (D > 0 && (ew = scan_rows(s, s->V, s->Cex, D, K1, st)) != IVX_OK) return ew;
                        k_cp_e<<<GQ, NT, 0, st>>>(s->Q, s->Cex, s->V, s->Aex, s->DT, s->GB, s->ZB, K1, D, s->Mdev,
                                                  fpp0, theta, s->E);
                        LB_HIP(hipGetLastError());
                        if ((ew = scan_rows(s, s->E, s->Eex, 1, K1, st)) != IVX_OK) return ew;
                        k_set_int<<<1, 64, 0, st>>>(s->Jdev, (int)(K1 - 1));
                        k_cp_find<<<GK, NT, 0, st>>>(s->Eex, s->Aex, s->DT, K1, fp0, fpp0, s->Jdev);
                        const uint64_t q = ++s->seq;
                        k_cp_gather<<<1, 64, 0, st>>>(s->Jdev, s->Pex, s->Cex, s->Eex, s->Aex, s->key2, K1, D, p0v,
                                                      fp0, fpp0, s->host_dev + OFF, flag_dev(s), q);
                        LB_HIP(hipGetLastError());
                        if ((ew = wait_published(s, q, st)) != IVX_OK) return ew;
                        f1 = h[OFF + 2 * D];
                        f2 = std::max(h[OFF + 2 * D + 1], EPS * fpp0);
                        told = h[OFF + 2 * D + 2];
                        J = (int64_t)h[OFF + 2 * D + 3];
                        return IVX_OK;
                    };
                    // First the breakpoints below a sampled threshold, sorted in one workgroup (an
                    // exact prefix of the full order; the minimiser usually lies within the first
                    // few segments).  A segment found inside the prefix is the full walk's
                    // segment; the prefix's closing segment is exact only when it holds every
                    // breakpoint.  Otherwise (or when the prefix overflows) sort them all.
                    bool done = false;
                    if (!opt.full_sort && n <= SEL_MAX_N) {
                    const uint64_t q = ++s->seq;
                    k_cp_select<<<1, SEL_NT, 0, st>>>(reinterpret_cast<const uint64_t *>(s->key), n, K,
                                                      reinterpret_cast<uint64_t *>(s->key2),
                                                      reinterpret_cast<uint32_t *>(s->val2), s->host_dev + SEL_OUT,
                                                      flag_dev(s), q);
                    LB_HIP(hipGetLastError());
                    {
                        const ivx_status es = wait_published(s, q, st);
                        if (es != IVX_OK) return es;
                    }
                    const double cs = h[SEL_OUT];
                    if (cs >= 0.0) {
                        const int64_t Kw = (int64_t)cs;
                        if ((e = walk(Kw)) != IVX_OK) return e;
                        done = J < Kw || Kw == K;
                    }
                    }
                    if (!done) {
                        ++nwalk_full;
                        // breakpoints t >= 0 (or +inf): their IEEE bit patterns order as the values
                        LB_HIP(radix_sort(s->sort_tmp, s->sort_bytes, reinterpret_cast<const uint64_t *>(s->key),
                                          reinterpret_cast<uint64_t *>(s->key2), reinterpret_cast<const uint32_t *>(s->val),
                                          reinterpret_cast<uint32_t *>(s->val2), (int)n, 64, st));
                        if ((e = walk(K)) != IVX_OK) return e;
                    }
                    const double dtm = std::max(-f1 / f2, 0.0);
                    tc = told + dtm;
                    for (int j = 0; j < D; ++j) c[j] = h[OFF + D + j] + dtm * h[OFF + j];
                    if (J > 0) {
                        const unsigned GJ = (unsigned)std::min<int64_t>(4096, (J + NT - 1) / NT);
                        k_cp_fix<<<GJ, NT, 0, st>>>(s->Jdev, s->val2, s->fixed);
                        LB_HIP(hipGetLastError());
                    }
                    nfixed += J;
                }
            }
            k_cp_xc<<<G, NT, 0, st>>>(s->x, s->d, s->fixed, tc, n, s->xc);
            LB_HIP(hipGetLastError());
            // ---- subspace minimisation
            const double *xbar = s->xc;
            if (k > 0 && nfixed < n) {
                Half mcy{}, mcs{};
                for (int a = 0; a < D; ++a) {
                    double v = 0.0;
                    for (int b = 0; b < D; ++b) v += mem.M[a * D + b] * c[b];
                    if (a < k) mcy.v[a] = v;
                    else mcs.v[a - k] = v;
                }
                // W^T r and the Gram matrix of the free rows are independent: both kernels and
                // both finishers, then one wait for the host (results land side by side)
                const int np = D * (D + 1) / 2;
                k_ss_r<<<G, NT, 0, st>>>(s->x, s->xc, s->g, s->fixed, s->S, s->Y, n, sl, theta, mcy, mcs, s->r,
                                         s->part + PART_R);
                k_ss_gram<<<G, NT, 0, st>>>(s->fixed, s->S, s->Y, n, sl, s->part);
                // both publish (the first one's stores are fenced too); the host waits for the second
                const uint64_t q1 = ++s->seq, q2 = ++s->seq;
                k_finish<<<1, FIN_NT, 0, st>>>(s->part + PART_R, (int)G, MAXD, MAXD, s->host_dev + OFF, nullptr, 0,
                                               nullptr, flag_dev(s), q1);
                k_finish<<<1, FIN_NT, 0, st>>>(s->part, (int)G, np, np, s->host_dev + OFF + MAXD, nullptr, 0, nullptr,
                                               flag_dev(s), q2);
                LB_HIP(hipGetLastError());
                {
                    const ivx_status es = wait_published(s, q2, st);
                    if (es != IVX_OK) return es;
                }
                std::vector<double> bvec(D);
                for (int j = 0; j < k; ++j) {
                    bvec[j] = h[OFF + j];
                    bvec[k + j] = theta * h[OFF + MAXM + j];
                }
                std::vector<double> A((size_t)D * D);
                for (int a = 0, q = 0; a < D; ++a)
                    for (int b = a; b < D; ++b, ++q) {
                        const double sa = a < k ? 1.0 : theta, sb = b < k ? 1.0 : theta;
                        A[a * D + b] = A[b * D + a] = sa * sb * h[OFF + MAXD + q];
                    }
                // N u = v with N = I - M A / theta, v = M b
                std::vector<double> N((size_t)D * D), v(D);
                for (int a = 0; a < D; ++a) {
                    double va = 0.0;
                    for (int b = 0; b < D; ++b) {
                        double ma = 0.0;
                        for (int q = 0; q < D; ++q) ma += mem.M[a * D + q] * A[q * D + b];
                        N[a * D + b] = (a == b ? 1.0 : 0.0) - ma / theta;
                        va += mem.M[a * D + b] * bvec[b];
                    }
                    v[a] = va;
                }
                if (!solve_dense(N, v, D, 1)) {
                    mem.reset(m);
                    std::fill(used.begin(), used.end(), 0);
                    mem.spare = 0;
                    continue;
                }
                Half uy{}, us{};
                for (int j = 0; j < k; ++j) {
                    uy.v[j] = v[j];
                    us.v[j] = v[k + j];
                }
                k_ss_du<<<G, NT, 0, st>>>(s->x, s->xc, s->g, s->r, s->fixed, s->S, s->Y, n, sl, theta, uy, us, pos,
                                          s->du, s->xbar, s->part);
                LB_HIP(hipGetLastError());
                if ((e = reduce_to_host(s, G, 2, 1, OFF, st)) != IVX_OK) return e;
                if (!(h[OFF] < 0.0)) {
                    const double alpha = std::min(1.0, h[OFF + 1]);
                    k_ss_trunc<<<G, NT, 0, st>>>(s->xc, s->du, s->fixed, alpha, n, s->xbar);
                    LB_HIP(hipGetLastError());
                }
                xbar = s->xbar;
            }
            // ---- line search along d = xbar - x
            k_dir<<<G, NT, 0, st>>>(s->x, xbar, s->g, n, pos, s->d, s->part);
            LB_HIP(hipGetLastError());
            if ((e = reduce_to_host(s, G, 3, 2, OFF, st)) != IVX_OK) return e;
            const double dnorm2 = h[OFF], gd0 = h[OFF + 1], rmin = h[OFF + 2];
            bool ok = gd0 < 0.0;
            double ft = 0.0, pgt = 0.0;
            if (ok) {
                WolfeSearch ls;
                double stp;
                if (nit == 0) {
                    ls.stpmax = 1.0;
                    stp = std::min(1.0 / std::sqrt(dnorm2), 1.0);
                } else {
                    ls.stpmax = std::max(std::min(rmin, 1e10), 1.0);
                    stp = 1.0;
                }
                ls.start(f, gd0, stp);
                int evals = 0;
                for (;;) {
                    k_trial<<<G, NT, 0, st>>>(s->x, s->d, xbar, ls.stp, ls.stp == 1.0 ? 1 : 0, n, s->xt, s->sky);
                    LB_HIP(hipGetLastError());
                    double gdt;
                    if ((e = evaluate(s->xt, s->d, s->gt, ft, gdt, pgt)) != IVX_OK) return e;
                    ++evals;
                    if (ft <= opt.target) break;
                    const int r = ls.next(ft, gdt);
                    if (r != 0) break;
                    if (evals >= opt.maxls || nfev >= opt.maxfun) {
                        ok = false;
                        break;
                    }
                }
            }
            if (ok && ft <= opt.target) {
                std::swap(s->x, s->xt);
                std::swap(s->g, s->gt);
                f = ft;
                pg = pgt;
                reason = IVX_LBFGSB_TARGET;
                break;
            }
            if (!ok) {
                if (nfev >= opt.maxfun) {
                    reason = IVX_LBFGSB_MAXFUN;
                    break;
                }
                if (k == 0) {
                    reason = IVX_LBFGSB_ABNORMAL;
                    break;
                }
                mem.reset(m);
                std::fill(used.begin(), used.end(), 0);
                mem.spare = 0;
                continue;
            }
            // ---- accept the step, update the memory
            const int spare = mem.spare;
            k_update<<<G, NT, 0, st>>>(s->x, s->xt, s->g, s->gt, n, pos, s->S, s->Y, spare, sl, s->part);
            LB_HIP(hipGetLastError());
            if ((e = reduce_to_host(s, G, UP_NS + 1, UP_NS, OFF, st)) != IVX_OK) return e;
            std::swap(s->x, s->xt);
            std::swap(s->g, s->gt);
            const double f_old = f;
            f = ft;
            pg = -h[OFF + UP_NS];
            ++nit;
            if (pg <= opt.gtol) {
                reason = IVX_LBFGSB_PGTOL;
                break;
            }
            if ((f_old - f) / std::max(std::max(std::fabs(f_old), std::fabs(f)), 1.0) <= opt.ftol) {
                reason = IVX_LBFGSB_FTOL;
                break;
            }
            if (nit >= opt.maxiter) {
                reason = IVX_LBFGSB_MAXITER;
                break;
            }
            if (nfev >= opt.maxfun) {
                reason = IVX_LBFGSB_MAXFUN;
                break;
            }
            const double sy = h[OFF], yy = h[OFF + 1], gs = h[OFF + 2], ss = h[OFF + 3];
            if (sy > EPS * (-gs)) {
                std::vector<double> sY(k), Sy(k), sS(k);
                for (int j = 0; j < k; ++j) {
                    sY[j] = h[OFF + 4 + j];
                    Sy[j] = h[OFF + 4 + MAXM + j];
                    sS[j] = h[OFF + 4 + 2 * MAXM + j];
                }
                int first = 0;
                if (mem.k == m) { // drop the oldest pair
                    used[mem.order[0]] = 0;
                    mem.order.erase(mem.order.begin());
                    for (int a = 0; a + 1 < m; ++a)
                        for (int b = 0; b + 1 < m; ++b) {
                            mem.SY[a][b] = mem.SY[a + 1][b + 1];
                            mem.SS[a][b] = mem.SS[a + 1][b + 1];
                        }
                    mem.k -= 1;
                    first = 1;
                }
                const int nw = mem.k;
                for (int j = first; j < k; ++j) {
                    const int b = j - first;
                    mem.SY[nw][b] = sY[j];
                    mem.SY[b][nw] = Sy[j];
                    mem.SS[nw][b] = mem.SS[b][nw] = sS[j];
                }
                mem.SY[nw][nw] = sy;
                mem.SS[nw][nw] = ss;
                mem.order.push_back(spare);
                used[spare] = 1;
                mem.k += 1;
                mem.spare = first_free();
                mem.theta = yy / sy;
                if (!mem.rebuild()) {
                    mem.reset(m);
                    std::fill(used.begin(), used.end(), 0);
                    mem.spare = 0;
                }
            }
        }
    }
    k_out<<<G, NT, 0, st>>>(s->x, n, xio);
    LB_HIP(hipGetLastError());
    LB_HIP(hipStreamSynchronize(st));
    res->f = f;
    res->pg_norm = pg;
    res->nit = nit;
    res->nfev = nfev;
    res->reason = reason;
    res->n_walks_full = (int32_t)std::min<int64_t>(nwalk_full, INT32_MAX);
    res->n_walks = nwalk;
    return IVX_OK;
}

} // extern "C"
