// Plan-time preparation of the visibilities on the device: flag compaction, Hermitian fold,
// fine-grid footprint coordinates and the stable sort into gridding tiles, one (pointing,
// channel) block at a time.
//
// The NUFFT spreads each visibility with a w x w kernel centred on its fine-grid position
// (Barnett et al. 2019, the paper's NUFFT reference, Sect. 2.1); only the fractional part of
// u * delta matters because the DFT of Sect. 2.1 is periodic in it, and a sample with u < 0
// is replaced by its Hermitian twin (-u, -v, conj(y)), which is valid for the real sky of
// Sect. 2.2.  Records of one block are ordered by (tile, caller index): the order, and so
// every sum the gridding pass forms, depends only on the data and the tile edge.
#include "ivx_internal.hpp"


namespace ivx {

namespace {

constexpr int BT = 256;

// Footprint of one visibility on the fine grid: start cell (row er0, column ec0) in the
// extended grid and the fractional offsets; returns whether the sample was folded.
__device__ __forceinline__ bool footprint(double u, double v, const BinGeom &b, int &er0, int &ec0, double &fx,
                                          double &fy) {
#pragma clang fp contract(off)
    const double ud = u * b.delta, vd = v * b.delta;
    double gx = (ud - floor(ud)) * b.nf;
    double gy = (vd - floor(vd)) * b.nf;
    if (gx >= b.nf) gx -= b.nf;
    if (gy >= b.nf) gy -= b.nf;
    const bool fold = gx > 0.5 * b.nf;
    if (fold) {
        gx = b.nf - gx;
        gy = b.nf - gy;
        if (gy >= b.nf) gy -= b.nf;
    }
    const double sx = gx - b.hw, sy = gy - b.hw;
    const double flx = floor(sx), fly = floor(sy);
    ec0 = (int)flx + 1 + b.O;
    er0 = (int)fly + 1 + b.O;
    fx = sx - flx;
    fy = sy - fly;
    return fold;
}

__device__ __forceinline__ VisCoord make_coord(int ix, int iy, double fx, double fy) {
#ifdef IVX_REAL_DOUBLE
    return VisCoord{(uint32_t)ix, (uint32_t)iy, fx, fy};
#else
    auto q24 = [](double f) -> uint32_t {
        double s = floor(f * 16777216.0 + 0.5);
        s = s > 16777215.0 ? 16777215.0 : s;
        s = s < 0.0 ? 0.0 : s;
        return (uint32_t)s;
    };
    return VisCoord{((uint32_t)ix << 24) | q24(fx), ((uint32_t)iy << 24) | q24(fy)};
#endif
}

__device__ __forceinline__ void coord_cells(const VisCoord &c, int &ix, int &iy) {
#ifdef IVX_REAL_DOUBLE
    ix = (int)c.ix;
    iy = (int)c.iy;
#else
    ix = (int)(c.xq >> 24);
    iy = (int)(c.yq >> 24);
#endif
}

// fractional offsets of a record
__device__ __forceinline__ void coord_fracs(const VisCoord &c, double &fx, double &fy) {
#ifdef IVX_REAL_DOUBLE
    fx = c.fx;
    fy = c.fy;
#else
    fx = (double)(c.xq & 0xFFFFFFu) * 5.9604644775390625e-08; // 2^-24
    fy = (double)(c.yq & 0xFFFFFFu) * 5.9604644775390625e-08;
#endif
}

__device__ __forceinline__ VisCoord move_coord(const VisCoord &c, int ix, int iy) {
#ifdef IVX_REAL_DOUBLE
    return VisCoord{(uint32_t)ix, (uint32_t)iy, c.fx, c.fy};
#else
    return VisCoord{((uint32_t)ix << 24) | (c.xq & 0xFFFFFFu), ((uint32_t)iy << 24) | (c.yq & 0xFFFFFFu)};
#endif
}

// live count of one block: visibilities whose flag is zero
__global__ __launch_bounds__(BT) void k_count_live(const uint8_t *__restrict__ flags, int64_t n,
                                                   unsigned long long *__restrict__ out) {
    __shared__ unsigned int sh[BT / 64];
    unsigned int c = 0;
    for (int64_t j = (int64_t)blockIdx.x * BT + threadIdx.x; j < n; j += (int64_t)gridDim.x * BT) c += flags[j] == 0;
    for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0;
        for (int i = 0; i < BT / 64; ++i) s += sh[i];
        atomicAdd(out, s);
    }
}

// Sort key of every sample of one block: (tile << 32) | caller index, or all ones for a
// flagged sample.  bad[0] / bad[1] receive the smallest global index of a non-finite
// sample / a negative weight.
__global__ __launch_bounds__(BT) void k_bin_keys(int64_t n, const real *__restrict__ uv, double scale,
                                                 const real *__restrict__ vis, const real *__restrict__ w,
                                                 const uint8_t *__restrict__ flags, BinGeom b, int64_t gbase,
                                                 uint64_t *__restrict__ keys, unsigned long long *__restrict__ bad) {
    const int64_t j = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (j >= n) return;
    uint64_t key = ~0ull;
    if (!(flags && flags[j])) {
        const double u = (double)uv[2 * j] * scale, v = (double)uv[2 * j + 1] * scale;
        const double yr = (double)vis[2 * j], yi = (double)vis[2 * j + 1], ww = (double)w[j];
        if (!isfinite(u) || !isfinite(v) || !isfinite(yr) || !isfinite(yi) || !isfinite(ww)) {
            atomicMin(&bad[0], (unsigned long long)(gbase + j));
        } else if (ww < 0.0) {
            atomicMin(&bad[1], (unsigned long long)(gbase + j));
        } else {
            int er0, ec0;
            double fx, fy;
            (void)footprint(u, v, b, er0, ec0, fx, fy);
            const uint32_t tile = (uint32_t)((er0 / b.T) * b.ntx + ec0 / b.T);
            key = ((uint64_t)tile << 32) | (uint64_t)j;
        }
    }
    keys[j] = key;
}

// Records of the sorted live samples of one block (n = its live count).
__global__ __launch_bounds__(BT) void k_bin_emit(int64_t n, const uint64_t *__restrict__ keys,
                                                 const real *__restrict__ uv, double scale,
                                                 const real *__restrict__ vis, const real *__restrict__ w,
                                                 BinGeom b, VisCoord *__restrict__ crd, cpx *__restrict__ svis,
                                                 real *__restrict__ swgt, int32_t *__restrict__ perm,
                                                 int32_t *__restrict__ counts) {
    const int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (i >= n) return;
    const uint64_t key = keys[i];
    if (key == ~0ull) return; // only after a bad sample, which fails the whole build
    const int64_t j = (int64_t)(uint32_t)key;
    const int tile = (int)(key >> 32);
    const double u = (double)uv[2 * j] * scale, v = (double)uv[2 * j + 1] * scale;
    int er0, ec0;
    double fx, fy;
    const bool fold = footprint(u, v, b, er0, ec0, fx, fy);
    const int ty = tile / b.ntx, tx = tile - ty * b.ntx;
    crd[i] = make_coord(ec0 - tx * b.T, er0 - ty * b.T, fx, fy);
    const real yi = vis[2 * j + 1];
    svis[i] = cpx{vis[2 * j], fold ? -yi : yi};
    swgt[i] = w[j];
    perm[i] = fold ? ~(int32_t)j : (int32_t)j;
    atomicAdd(&counts[tile], 1);
}

// Re-keying of one block's records for another tile edge: footprint start recovered from
// the old tile (found in the block's old tile prefix) and the tile-relative cell.
__global__ __launch_bounds__(BT) void k_rekey(int64_t n, const VisCoord *__restrict__ crd,
                                              const int32_t *__restrict__ perm, const int32_t *__restrict__ tstart,
                                              int ntiles_old, int ntx_old, int T_old, int ntx_new, int T_new,
                                              uint64_t *__restrict__ keys, uint32_t *__restrict__ vals,
                                              int2 *__restrict__ foot, Regeom rg, double2 *__restrict__ frac) {
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (i >= n) return;
    int lo = 0, hi = ntiles_old - 1; // last tile t with tstart[t] <= i
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tstart[mid] <= (int32_t)i) lo = mid;
        else hi = mid - 1;
    }
    int ix, iy;
    coord_cells(crd[i], ix, iy);
    const int ty = lo / ntx_old, tx = lo - ty * ntx_old;
    int er0 = ty * T_old + iy, ec0 = tx * T_old + ix;
    if (frac) {
        // fine-grid position under the old geometry, scaled to the new grid, split for the new width
        double fx, fy;
        coord_fracs(crd[i], fx, fy);
        const double gx = ((double)(ec0 - 1 - rg.O_old) + fx + rg.hw_old) * rg.ratio;
        const double gy = ((double)(er0 - 1 - rg.O_old) + fy + rg.hw_old) * rg.ratio;
        const double sx = gx - rg.hw_new, sy = gy - rg.hw_new;
        const double flx = floor(sx), fly = floor(sy);
        ec0 = (int)flx + 1 + rg.O_new;
        er0 = (int)fly + 1 + rg.O_new;
        frac[i] = double2{sx - flx, sy - fly};
    }
    const uint32_t tile = (uint32_t)((er0 / T_new) * ntx_new + ec0 / T_new);
    const int32_t p = perm[i];
    const uint32_t src = (uint32_t)(p < 0 ? ~p : p);
    keys[i] = ((uint64_t)tile << 32) | src;
    vals[i] = (uint32_t)i;
    foot[i] = int2{er0, ec0};
}

__global__ __launch_bounds__(BT) void k_rebin_emit(int64_t n, const uint64_t *__restrict__ keys,
                                                   const uint32_t *__restrict__ vals, const int2 *__restrict__ foot,
                                                   const VisCoord *__restrict__ crd, const cpx *__restrict__ vis,
                                                   const real *__restrict__ wgt, const int32_t *__restrict__ perm,
                                                   int ntx, int T, VisCoord *__restrict__ crd_o,
                                                   cpx *__restrict__ vis_o, real *__restrict__ wgt_o,
                                                   int32_t *__restrict__ perm_o, int32_t *__restrict__ counts,
                                                   const double2 *__restrict__ frac) {
    const int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (i >= n) return;
    const uint32_t o = vals[i];
    const int tile = (int)(keys[i] >> 32);
    const int ty = tile / ntx, tx = tile - ty * ntx;
    const int2 f = foot[o];
    if (frac) crd_o[i] = make_coord(f.y - tx * T, f.x - ty * T, frac[o].x, frac[o].y);
    else crd_o[i] = move_coord(crd[o], f.y - tx * T, f.x - ty * T);
    vis_o[i] = vis[o];
    wgt_o[i] = wgt[o];
    perm_o[i] = perm[o];
    atomicAdd(&counts[tile], 1);
}

// Data update of one block in sorted order: svis[s] = vis[perm[s]] (conjugated when
// folded), swgt[s] = w[perm[s]] when w is given; bad[0] is set on a non-finite value or a
// negative weight.
__global__ __launch_bounds__(BT) void k_gather_block(int64_t n, const int32_t *__restrict__ perm,
                                                     const real *__restrict__ vis, const real *__restrict__ w,
                                                     cpx *__restrict__ svis, real *__restrict__ swgt,
                                                     unsigned int *__restrict__ bad) {
    const int64_t s = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (s >= n) return;
    const int32_t p = perm[s];
    const int64_t src = p < 0 ? ~p : p;
    cpx y{vis[2 * src], vis[2 * src + 1]};
    if (p < 0) y.im = -y.im;
    bool ok = isfinite(y.re) && isfinite(y.im);
    svis[s] = y;
    if (w) {
        const real ww = w[src];
        ok = ok && isfinite(ww) && ww >= real(0);
        swgt[s] = ww;
    }
    if (!ok) bad[0] = 1u;
}

unsigned grid1(int64_t n) { return (unsigned)((n + BT - 1) / BT); }

} // namespace

hipError_t launch_count_live(const uint8_t *flags, int64_t n, unsigned long long *out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const unsigned nb = (unsigned)std::min<int64_t>((n + BT - 1) / BT, 1024);
    k_count_live<<<nb, BT, 0, st>>>(flags, n, out);
    return hipGetLastError();
}

hipError_t launch_bin_keys(int64_t n, const real *uv, double scale, const real *vis, const real *w,
                           const uint8_t *flags, const BinGeom &b, int64_t gbase, uint64_t *keys,
                           unsigned long long *bad, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_bin_keys<<<grid1(n), BT, 0, st>>>(n, uv, scale, vis, w, flags, b, gbase, keys, bad);
    return hipGetLastError();
}

hipError_t launch_bin_emit(int64_t n, const uint64_t *keys, const real *uv, double scale, const real *vis,
                           const real *w, const BinGeom &b, VisCoord *crd, cpx *svis, real *swgt, int32_t *perm,
                           int32_t *counts, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_bin_emit<<<grid1(n), BT, 0, st>>>(n, keys, uv, scale, vis, w, b, crd, svis, swgt, perm, counts);
    return hipGetLastError();
}

hipError_t launch_rekey(int64_t n, const VisCoord *crd, const int32_t *perm, const int32_t *tstart, int ntiles_old,
                        int ntx_old, int T_old, int ntx_new, int T_new, uint64_t *keys, uint32_t *vals, int2 *foot,
                        hipStream_t st, const Regeom *rg, double2 *frac) {
    if (n <= 0) return hipSuccess;
    if ((rg == nullptr) != (frac == nullptr)) return hipErrorInvalidValue;
    const Regeom r = rg ? *rg : Regeom{1.0, 0.0, 0.0, 0, 0};
    k_rekey<<<grid1(n), BT, 0, st>>>(n, crd, perm, tstart, ntiles_old, ntx_old, T_old, ntx_new, T_new, keys, vals,
                                     foot, r, frac);
    return hipGetLastError();
}

hipError_t launch_rebin_emit(int64_t n, const uint64_t *keys, const uint32_t *vals, const int2 *foot,
                             const VisCoord *crd, const cpx *vis, const real *wgt, const int32_t *perm, int ntx,
                             int T, VisCoord *crd_o, cpx *vis_o, real *wgt_o, int32_t *perm_o, int32_t *counts,
                             hipStream_t st, const double2 *frac) {
    if (n <= 0) return hipSuccess;
    k_rebin_emit<<<grid1(n), BT, 0, st>>>(n, keys, vals, foot, crd, vis, wgt, perm, ntx, T, crd_o, vis_o, wgt_o,
                                          perm_o, counts, frac);
    return hipGetLastError();
}

hipError_t launch_gather_block(int64_t n, const int32_t *perm, const real *vis, const real *w, cpx *svis,
                               real *swgt, unsigned int *bad, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_gather_block<<<grid1(n), BT, 0, st>>>(n, perm, vis, w, svis, swgt, bad);
    return hipGetLastError();
}

hipError_t sort_keys(void *temp, size_t &temp_bytes, const uint64_t *in, uint64_t *out, int n, int end_bit,
                     hipStream_t st) {
    if (!temp) {
        temp_bytes = radix_sort_temp_bytes(n, false);
        return hipSuccess;
    }
    return radix_sort(temp, temp_bytes, in, out, nullptr, nullptr, n, end_bit, st);
}

hipError_t sort_pairs(void *temp, size_t &temp_bytes, const uint64_t *kin, uint64_t *kout, const uint32_t *vin,
                      uint32_t *vout, int n, int end_bit, hipStream_t st) {
    if (!temp) {
        temp_bytes = radix_sort_temp_bytes(n, true);
        return hipSuccess;
    }
    return radix_sort(temp, temp_bytes, kin, kout, vin, vout, n, end_bit, st);
}

} // namespace ivx
