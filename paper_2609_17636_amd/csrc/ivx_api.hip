// C ABI of the Classic3D objective/gradient engine: plan creation, plan-time data
// preparation (Sect. 3.2 concatenation of all pointings; flag compaction; Hermitian fold;
// tile binning), evaluation sequencing on a HIP stream, and error reporting.
#include "ivx_internal.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

using namespace ivx;

namespace {

thread_local std::string g_last_error;

ivx_status fail(ivx_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}

ivx_status hip_fail(hipError_t e, const char *where) {
    return fail(IVX_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

} // namespace

namespace ivx {
// Error reporting shared with the warm-start network (same thread-local message).
ivx_status set_error(ivx_status s, const std::string &msg) { return fail(s, msg); }
} // namespace ivx

namespace {

#define IVX_HIP(call)                                        \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return hip_fail(e_, #call);    \
    } while (0)

// ------------------------------------------------------------- kernel mathematics
// Exponential of semicircle, phi(z) = exp(beta (sqrt(1 - (2z/W)^2) - 1)), |z| <= W/2
// (Barnett, Magland & af Klinteberg 2019).
double es_phi(double z, double W, double beta) {
    const double t = 2.0 * z / W;
    const double q = 1.0 - t * t;
    if (q < 0.0) return 0.0;
    return std::exp(beta * (std::sqrt(q) - 1.0));
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration on P_n).
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            const double dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        const double dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// Fourier transform of the kernel at angular frequency kappa (grid units):
// phi_hat(kappa) = int_{-W/2}^{W/2} phi(z) cos(kappa z) dz.
double es_phihat(double kappa, double W, double beta, const std::vector<double> &x,
                 const std::vector<double> &w) {
    double s = 0.0;
    for (size_t i = 0; i < x.size(); ++i) {
        const double z = 0.5 * W * x[i];
        s += w[i] * es_phi(z, W, beta) * std::cos(kappa * z);
    }
    return 0.5 * W * s;
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

} // namespace

struct ivx_plan {
    ivx_problem d{};
    std::vector<int64_t> offsets;
    std::vector<double> fscale;
    Geom g{};
    double beta = 0.0;
    int nwave = 4;
    int lanes = 16;
    int vpi = 2;
    int chunk_max = 256;
    int occupancy = GRIDMX_OCC_AUTO; // matrix-core gridder register budget (waves per SIMD)
    int fused_fold = 1;              // slot fold inside the inverse column pass: 0 never, 1 when it pays, 2 always
    // every call that reuses the evaluation buffers advances the epoch; ivx_objective_backward
    // needs the buffers exactly as ivx_objective_forward left them
    uint64_t epoch = 0, fwd_epoch = ~0ull;
    const void *fwd_sky = nullptr;
    int tile_fixed = 0;
    std::vector<real> dq_host;
    std::vector<cpx> tw_host;
    bool has_data = false;
    int64_t m_total = 0, m_live = 0;
    int n_work = 0, n_slots = 0;
    int sd_rb = 0;
    std::vector<real> gB_host;
    std::vector<int64_t> block_live;  // live count prefix per block
    bool shared_uv = false;           // uv and weights given once per pointing
    std::vector<int64_t> pt_off;      // shared_uv: pointing offsets into uv / weights
    // tiling the records are currently sorted for, and their per-(block, tile) counts
    int bin_T = 0, bin_ntx = 0, bin_ntiles = 0;
    int bin_W = 0, bin_nf = 0;        // kernel width and fine grid the records are binned for
    bool geometry_auto = false;       // W and n_f chosen by the library (the autotuner may change them)
    double eps_target = 0.0;          // accuracy the autotuner's geometries must reach
    std::vector<int32_t> tcount;      // [n_items][bin_ntiles]
    // device memory
    std::vector<DevBuf> bufs;
    real *d_dq = nullptr, *d_fscale = nullptr;
    cpx *d_tw = nullptr;
    real *d_beams = nullptr, *d_interp = nullptr;
    VisCoord *d_crd = nullptr;
    cpx *d_vis = nullptr;
    real *d_wgt = nullptr;
    int32_t *d_perm = nullptr;   // caller index within the block (bit-inverted when folded)
    int64_t *d_boff = nullptr;   // caller offset of each block
    int32_t *d_tstart = nullptr; // [n_items][bin_ntiles + 1] tile prefix of each block's records
    WorkItem *d_work = nullptr;
    int32_t *d_tslot = nullptr;
    cpx *d_R = nullptr, *d_ext = nullptr, *d_slots = nullptr;
    real *d_gp = nullptr;
    int32_t *d_cptr = nullptr; // reprojection transpose: slice offsets (sliced layout)
    CsrEnt *d_cent = nullptr;  // and entries
    real *d_sdmap = nullptr, *d_gB = nullptr, *d_U = nullptr, *d_E = nullptr;
    double *d_jpart = nullptr, *d_rpart = nullptr, *d_kpart = nullptr, *d_terms = nullptr;
    double *d_npart = nullptr; // spectral-term partial per sky block
    int n_rpart = 0, n_kpart = 0;
    size_t dev_bytes = 0;
    // per-tile device arrays that depend on the tile size
    size_t tile_bytes = 0;
    // stage timing
    uint32_t timing_mask = 0;
    std::vector<hipEvent_t> ev_pool;            // all events ever created (reused)
    std::vector<std::pair<int, int>> ev_used;   // (stage, index of start event) pending
    size_t ev_next = 0;
    int64_t timed_evals = 0;
    // one captured evaluation, replayed while (sky, grad) stay the same
    bool use_graph = true;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec = nullptr;
    const void *g_sky = nullptr;
    void *g_grad = nullptr;
    double *g_terms = nullptr;
    int64_t graph_nodes = 0;
    // full forward model (w-stacked planes); set by ivx_plan_set_w, dropped by set_data
    bool w_on = false;
    int w_W = 0;                      // w kernel width in planes
    double w_sigma = 2.0, w_beta = 0.0, w_dw = 0.0, w_xc = 0.0, w_X = 0.0;
    int w_planes = 0;                 // planes of the block with the widest w range
    uint64_t work_version = 0;        // advanced by every new work list
    uint64_t w_version = ~0ull;       // work list the plane coordinates were sorted for
    std::vector<double> uv_scale;     // shared uv: the channel scales of the caller's tracks
    std::vector<double> w0_host;
    std::vector<int32_t> np_host;
    real *d_wsrc = nullptr;           // the caller's w, caller layout
    WZ *d_wz = nullptr;               // plane coordinate of every record
    cpx *d_wacc = nullptr;            // per-record plane accumulator / adjoint coefficient
    cpx *d_wR = nullptr;              // row-pass buffer of the planes
    size_t wR_count = 0;
    double *d_wxp = nullptr, *d_wtp = nullptr;
    real *d_wcorr = nullptr;
    double *d_w0 = nullptr;
    int32_t *d_wnp = nullptr;
    int32_t *d_wcnt = nullptr;        // per-work-item record counts below each half plane (or NULL)
    uint8_t *d_wsact = nullptr;       // adjoint plane pass: slot windows written (1) or skipped (0)
    int wsact_count = 0;
    int wncnt = 0;
};

namespace {

template <typename T> ivx_status dalloc(ivx_plan *p, T **out, size_t count) {
    *out = nullptr;
    if (count == 0) count = 1;
    void *ptr = nullptr;
    const size_t bytes = count * sizeof(T);
    hipError_t e = hipMalloc(&ptr, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(IVX_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    p->bufs.push_back(DevBuf{ptr, bytes});
    p->dev_bytes += bytes;
    *out = static_cast<T *>(ptr);
    return IVX_OK;
}

void drop_graph(ivx_plan *p) {
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    p->gexec = nullptr;
    p->g_sky = nullptr;
    p->g_grad = nullptr;
    p->g_terms = nullptr;
    p->graph_nodes = 0;
}

void free_all(ivx_plan *p) {
    drop_graph(p);
    for (auto &b : p->bufs) (void)hipFree(b.p);
    p->bufs.clear();
    p->dev_bytes = 0;
    p->d_dq = p->d_fscale = nullptr;
    p->d_tw = nullptr;
    p->d_beams = p->d_interp = nullptr;
    p->d_crd = nullptr;
    p->d_vis = nullptr;
    p->d_wgt = nullptr;
    p->d_perm = nullptr;
    p->d_boff = nullptr;
    p->d_tstart = nullptr;
    p->bin_T = p->bin_ntx = p->bin_ntiles = 0;
    p->bin_W = p->bin_nf = 0;
    p->tcount.clear();
    p->d_work = nullptr;
    p->d_tslot = nullptr;
    p->d_R = p->d_ext = p->d_slots = nullptr;
    p->d_gp = nullptr;
    p->d_cptr = nullptr;
    p->d_cent = nullptr;
    p->d_sdmap = p->d_gB = p->d_U = p->d_E = nullptr;
    p->d_jpart = p->d_rpart = p->d_kpart = p->d_terms = nullptr;
    p->d_npart = nullptr;
    p->has_data = false;
    p->w_on = false;
    p->w_version = ~0ull;
    p->w_planes = 0;
    p->d_wsrc = nullptr;
    p->d_wz = nullptr;
    p->d_wacc = p->d_wR = nullptr;
    p->wR_count = 0;
    p->d_wxp = p->d_wtp = nullptr;
    p->d_wcorr = nullptr;
    p->d_w0 = nullptr;
    p->d_wnp = nullptr;
    p->d_wcnt = nullptr;
    p->wncnt = 0;
    p->d_wsact = nullptr;
    p->wsact_count = 0;
}

void free_one(ivx_plan *p, void *ptr) {
    for (size_t i = 0; i < p->bufs.size(); ++i) {
        if (p->bufs[i].p == ptr) {
            (void)hipFree(ptr);
            p->dev_bytes -= p->bufs[i].bytes;
            p->bufs.erase(p->bufs.begin() + i);
            return;
        }
    }
}

// Column stride of a (column-major) gridding window in LDS, in complex cells.  A lane of a
// 16-lane group with W <= 8 reads column j, row h (j < 8, h < 2) of a footprint: with a
// stride of twice an odd number the 16 values j * ldw + h are distinct mod 16, i.e. the
// lanes hit distinct 8-byte bank pairs.  Other layouts walk up to 16 columns at one row:
// an odd stride spreads those.
int pick_ldw(int win, int W, int lanes) {
    if (lanes == 16 && W <= 8) return win + ((2 - win % 4) + 4) % 4;
    return win | 1;
}

// Geometry that depends on the tile edge.
void set_tile(ivx_plan *p, int T) {
    Geom &g = p->g;
    g.T = T;
    g.win = T + g.W - 1;
    g.ldw = pick_ldw(g.win, g.W, p->lanes);
    // footprint starts reach extended row nf + (O - W/2) + 1 and column nf/2 + 1 + ...
    const int max_er0 = g.nf + g.O; // generous upper bound on footprint-start rows
    const int max_ec0 = g.nf / 2 + g.O + 1;
    g.nty = max_er0 / T + 1;
    g.ntx = max_ec0 / T + 1;
    g.eh = g.nty * T + g.W - 1;
    g.ew = g.ntx * T + g.W - 1;
    g.ext_stride = (int64_t)g.eh * g.ew;
    g.win_stride = (int64_t)g.win * g.win;
}

bool tile_fits(const ivx_plan *p, int T, int nwave, int lanes) {
    if (T < p->g.W || T > 255) return false;
    if (lanes == GRID_MFMA_LANES) {
#ifdef IVX_REAL_DOUBLE
        return false; // the matrix-core gridder is float only
#else
        return nwave == 1 && T + p->g.W - 1 <= 16;
#endif
    }
    Geom g = p->g;
    g.T = T;
    g.win = T + g.W - 1;
    g.ldw = pick_ldw(g.win, g.W, lanes);
    if (lanes == 8 && g.W > 8) return false;
    return grid_lds_bytes(g, nwave, lanes) <= 80 * 1024; // two blocks per 160 KB compute unit
}

// NUFFT geometry: fine grid n_f, kernel width W, kernel shape beta (scaled from the 2.30 W of
// two-fold oversampling), deapodization 1 / phi_hat at the sub-image frequencies, twiddles.
void set_geometry_fields(ivx_plan *p, int W, int nf) {
    Geom &g = p->g;
    g.nf = nf;
    g.logn = ilog2(nf);
    g.rw = nf / 2 + 1;
    g.W = W;
    g.O = (W + 1) / 2;
    const double sigma = (double)nf / g.nk;
    p->beta = 2.30 * W * (1.0 - 1.0 / (2.0 * sigma)) / 0.75;
    g.beta = (real)p->beta;
    g.r_stride = (int64_t)g.nk * g.rw;
    g.hs_stride = (int64_t)g.nf * g.rw;
    std::vector<double> gx, gw;
    gauss_legendre(std::max(64, 8 * W), gx, gw);
    p->dq_host.resize(g.nk);
    for (int a = 0; a < g.nk; ++a) {
        const double kap = 2.0 * M_PI * (a - g.nk / 2) / nf;
        p->dq_host[a] = (real)(1.0 / es_phihat(kap, W, p->beta, gx, gw));
    }
    p->tw_host.resize(nf);
    for (int t = 0; t < nf; ++t) {
        const double th = -2.0 * M_PI * t / nf;
        p->tw_host[t] = cpx{(real)std::cos(th), (real)std::sin(th)};
    }
}

// Accuracy probe of a geometry: the largest error, over the sub-image's frequencies k and
// positions x in one fine cell, of the one-dimensional transform of a unit point source that
// the plan's spreading kernel and deapodization compute,
//   | dq(k) sum_t phi(x - t) exp(-2 pi i k t / n_f) - exp(-2 pi i k x / n_f) |,
// against its closed form (the second term).  A two-dimensional transform is separable, so
// its error is at most about twice this.
double nufft_probe_error(int nk, int nf, int W) {
    const double sigma = (double)nf / nk;
    const double beta = 2.30 * W * (1.0 - 1.0 / (2.0 * sigma)) / 0.75;
    std::vector<double> gx, gw;
    gauss_legendre(std::max(64, 8 * W), gx, gw);
    double worst = 0.0;
    const int nx = 33;
    std::vector<double> phi(W);
    for (int ix = 0; ix < nx; ++ix) {
        const double x = (double)ix / (nx - 1);
        const double t0 = std::floor(x - 0.5 * W) + 1.0;
        for (int t = 0; t < W; ++t) phi[t] = es_phi(x - (t0 + t), W, beta);
        for (int k = -nk / 2; k < nk / 2; ++k) {
            const double dq = 1.0 / es_phihat(2.0 * M_PI * k / nf, W, beta, gx, gw);
            double re = 0.0, im = 0.0;
            for (int t = 0; t < W; ++t) {
                const double th = -2.0 * M_PI * k * (t0 + t) / nf;
                re += phi[t] * std::cos(th);
                im += phi[t] * std::sin(th);
            }
            const double th = -2.0 * M_PI * k * x / nf;
            worst = std::max(worst, std::hypot(dq * re - std::cos(th), dq * im - std::sin(th)));
        }
    }
    return worst;
}

// Switch a plan with data to another fine grid / kernel width: new tables and row-FFT buffers
// (allocated before anything is released, so a failure leaves the plan as it was); the
// records are re-binned by the next build_bins.
ivx_status apply_geometry(ivx_plan *p, int W, int nf) {
    if (W == p->g.W && nf == p->g.nf) return IVX_OK;
    const int64_t n_items = (int64_t)p->g.C * p->g.P;
    cpx *tw = nullptr, *R = nullptr;
    ivx_status s;
    if ((s = dalloc(p, &tw, nf)) != IVX_OK) return s;
    if ((s = dalloc(p, &R, (size_t)n_items * p->g.nk * (nf / 2 + 1))) != IVX_OK) {
        free_one(p, tw);
        return s;
    }
    drop_graph(p);
    free_one(p, p->d_tw);
    free_one(p, p->d_R);
    p->d_tw = tw;
    p->d_R = R;
    set_geometry_fields(p, W, nf);
    IVX_HIP(hipMemcpy(p->d_dq, p->dq_host.data(), p->g.nk * sizeof(real), hipMemcpyHostToDevice));
    IVX_HIP(hipMemcpy(p->d_tw, p->tw_host.data(), nf * sizeof(cpx), hipMemcpyHostToDevice));
    ++p->epoch;
    return IVX_OK;
}

// Default blocking: the widest block (4 waves) and a 16-cell tile when they fit the LDS
// budget, else fewer waves, else other tile edges.  ivx_autotune refines it by timing.
bool auto_blocking(ivx_plan *p) {
    const int waves[] = {4, 2, 1};
    const int cand[] = {16, 24, 12, 32, 8};
    for (int nw : waves)
        for (int T : cand)
            if (tile_fits(p, T, nw, 16)) {
                p->nwave = nw;
                p->lanes = 16;
                set_tile(p, T);
                return true;
            }
    return false;
}

// Plan-time temporary device buffer (not counted in the plan's memory).
struct TmpBuf {
    void *p = nullptr;
    ~TmpBuf() {
        if (p) (void)hipFree(p);
    }
    hipError_t get(size_t bytes) {
        if (p) (void)hipFree(p);
        p = nullptr;
        return hipMalloc(&p, bytes > 0 ? bytes : 1);
    }
    template <typename T> T *as() const { return static_cast<T *>(p); }
};

bool on_device(const void *ptr) {
    if (!ptr) return false;
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, ptr) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

// The caller's visibility arrays.  Per block b = k * C + c: vis / flags at the block's
// caller offset; uv / weights at the same offset, or (shared_uv) at pointing k's offset,
// with uv multiplied by scale[c].
struct VisSource {
    const real *uv = nullptr, *vis = nullptr, *w = nullptr;
    const uint8_t *flags = nullptr;
    const double *scale = nullptr;
};

// One (possibly staged) array of a block: the caller's device pointer, or a copy of the
// caller's host data in `stage`.
template <typename T>
ivx_status block_view(const T *base, bool dev, int64_t off, int64_t count, const TmpBuf &stage, const T **out,
                      hipStream_t st) {
    if (dev || count == 0) {
        *out = base + off;
        return IVX_OK;
    }
    IVX_HIP(hipMemcpyAsync(stage.p, base + off, count * sizeof(T), hipMemcpyHostToDevice, st));
    *out = stage.as<T>();
    return IVX_OK;
}

int key_bits(int ntiles) {
    int b = 1;
    while ((1 << b) <= ntiles) ++b;
    return 32 + b;
}

// Record counts per (block, tile) -> host copy, and the per-block tile prefix on the device
// in `tstart` (a plan buffer of n_items * (ntiles + 1) entries that replaces the old one).
ivx_status store_counts(ivx_plan *p, const int32_t *d_counts, int ntiles, int32_t *tstart, hipStream_t st) {
    const int n_items = p->g.C * p->g.P;
    std::vector<int32_t> cnt((size_t)n_items * ntiles);
    IVX_HIP(hipMemcpyAsync(cnt.data(), d_counts, cnt.size() * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    IVX_HIP(hipStreamSynchronize(st));
    std::vector<int32_t> ts((size_t)n_items * (ntiles + 1));
    for (int b = 0; b < n_items; ++b) {
        int32_t acc = 0;
        for (int t = 0; t < ntiles; ++t) {
            ts[(size_t)b * (ntiles + 1) + t] = acc;
            acc += cnt[(size_t)b * ntiles + t];
        }
        ts[(size_t)b * (ntiles + 1) + ntiles] = acc;
        if (acc != p->block_live[b + 1] - p->block_live[b]) return fail(IVX_EHIP, "binning lost records");
    }
    if (p->d_tstart) free_one(p, p->d_tstart);
    p->d_tstart = tstart;
    IVX_HIP(hipMemcpyAsync(p->d_tstart, ts.data(), ts.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    IVX_HIP(hipStreamSynchronize(st));
    p->tcount.swap(cnt);
    p->bin_T = p->g.T;
    p->bin_ntx = p->g.ntx;
    p->bin_ntiles = ntiles;
    p->bin_W = p->g.W;
    p->bin_nf = p->g.nf;
    return IVX_OK;
}

// Live records of every block from the caller's arrays, sorted by (tile, caller index) for
// the current tile edge.  Fails with IVX_ENONFINITE / IVX_EINVAL at the first bad sample.
ivx_status bin_from_caller(ivx_plan *p, const VisSource &src, hipStream_t st) {
    const Geom &g = p->g;
    const int n_items = g.C * g.P;
    const int ntiles = g.nty * g.ntx;
    std::vector<int64_t> nb(n_items), live(n_items);
    int64_t maxn = 0, maxuv = 0;
    for (int b = 0; b < n_items; ++b) {
        nb[b] = p->offsets[b + 1] - p->offsets[b];
        if (nb[b] > (int64_t)INT32_MAX)
            return fail(IVX_EINVAL, "a (pointing, channel) block holds more than 2^31 - 1 visibilities");
        maxn = std::max(maxn, nb[b]);
    }
    if (p->shared_uv)
        for (int k = 0; k < g.P; ++k) maxuv = std::max(maxuv, p->pt_off[k + 1] - p->pt_off[k]);
    else
        maxuv = maxn;
    const bool uv_dev = on_device(src.uv), vis_dev = on_device(src.vis), w_dev = on_device(src.w);
    const bool fl_dev = on_device(src.flags);
    // ---- live counts (from the flags alone)
    if (!src.flags) {
        live = nb;
    } else if (fl_dev) {
        TmpBuf dc;
        IVX_HIP(dc.get(n_items * sizeof(unsigned long long)));
        IVX_HIP(hipMemsetAsync(dc.p, 0, n_items * sizeof(unsigned long long), st));
        for (int b = 0; b < n_items; ++b)
            IVX_HIP(launch_count_live(src.flags + p->offsets[b], nb[b], dc.as<unsigned long long>() + b, st));
        std::vector<unsigned long long> h(n_items);
        IVX_HIP(hipMemcpyAsync(h.data(), dc.p, n_items * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
        IVX_HIP(hipStreamSynchronize(st));
        for (int b = 0; b < n_items; ++b) live[b] = (int64_t)h[b];
    } else {
        for (int b = 0; b < n_items; ++b)
            live[b] = (int64_t)std::count(src.flags + p->offsets[b], src.flags + p->offsets[b + 1], (uint8_t)0);
    }
    p->block_live.assign(n_items + 1, 0);
    for (int b = 0; b < n_items; ++b) p->block_live[b + 1] = p->block_live[b] + live[b];
    p->m_live = p->block_live[n_items];
    ivx_status s;
    const size_t L = (size_t)std::max<int64_t>(p->m_live, 1);
    if ((s = dalloc(p, &p->d_crd, L)) != IVX_OK || (s = dalloc(p, &p->d_vis, L)) != IVX_OK ||
        (s = dalloc(p, &p->d_wgt, L)) != IVX_OK || (s = dalloc(p, &p->d_perm, L)) != IVX_OK)
        return s;
    // ---- temporaries
    const int end_bit = key_bits(ntiles);
    size_t sort_bytes = 0;
    IVX_HIP(sort_keys(nullptr, sort_bytes, nullptr, nullptr, (int)std::max<int64_t>(maxn, 1), end_bit, st));
    TmpBuf keys, keys2, temp, counts, bad, s_uv, s_vis, s_w, s_fl;
    IVX_HIP(keys.get(maxn * sizeof(uint64_t)));
    IVX_HIP(keys2.get(maxn * sizeof(uint64_t)));
    IVX_HIP(temp.get(sort_bytes));
    IVX_HIP(counts.get((size_t)n_items * ntiles * sizeof(int32_t)));
    IVX_HIP(bad.get(2 * sizeof(unsigned long long)));
    if (!uv_dev) IVX_HIP(s_uv.get(2 * maxuv * sizeof(real)));
    if (!w_dev) IVX_HIP(s_w.get(maxuv * sizeof(real)));
    if (!vis_dev) IVX_HIP(s_vis.get(2 * maxn * sizeof(real)));
    if (src.flags && !fl_dev) IVX_HIP(s_fl.get(maxn));
    int32_t *tstart = nullptr;
    if ((s = dalloc(p, &tstart, (size_t)n_items * (ntiles + 1))) != IVX_OK) return s;
    IVX_HIP(hipMemsetAsync(counts.p, 0, (size_t)n_items * ntiles * sizeof(int32_t), st));
    IVX_HIP(hipMemsetAsync(bad.p, 0xFF, 2 * sizeof(unsigned long long), st));
    const BinGeom bg{p->d.pixel_rad, (double)g.nf, 0.5 * g.W, g.O, g.T, g.ntx};
    int staged_k = -1;
    const real *uvb = nullptr, *wb = nullptr;
    for (int b = 0; b < n_items; ++b) {
        if (nb[b] == 0) continue;
        const int k = b / g.C, c = b - (b / g.C) * g.C;
        const int64_t off = p->offsets[b];
        double scale = 1.0;
        if (p->shared_uv) {
            scale = src.scale[c];
            if (k != staged_k) {
                const int64_t po = p->pt_off[k], pn = p->pt_off[k + 1] - p->pt_off[k];
                if ((s = block_view(src.uv, uv_dev, 2 * po, 2 * pn, s_uv, &uvb, st)) != IVX_OK ||
                    (s = block_view(src.w, w_dev, po, pn, s_w, &wb, st)) != IVX_OK)
                    return s;
                staged_k = k;
            }
        } else if ((s = block_view(src.uv, uv_dev, 2 * off, 2 * nb[b], s_uv, &uvb, st)) != IVX_OK ||
                   (s = block_view(src.w, w_dev, off, nb[b], s_w, &wb, st)) != IVX_OK) {
            return s;
        }
        const real *vb = nullptr;
        const uint8_t *fb = nullptr;
        if ((s = block_view(src.vis, vis_dev, 2 * off, 2 * nb[b], s_vis, &vb, st)) != IVX_OK) return s;
        if (src.flags && (s = block_view(src.flags, fl_dev, off, nb[b], s_fl, &fb, st)) != IVX_OK) return s;
        IVX_HIP(launch_bin_keys(nb[b], uvb, scale, vb, wb, fb, bg, off, keys.as<uint64_t>(),
                                bad.as<unsigned long long>(), st));
        size_t tb = sort_bytes;
        IVX_HIP(sort_keys(temp.p, tb, keys.as<uint64_t>(), keys2.as<uint64_t>(), (int)nb[b], end_bit, st));
        const int64_t L0 = p->block_live[b];
        IVX_HIP(launch_bin_emit(live[b], keys2.as<uint64_t>(), uvb, scale, vb, wb, bg, p->d_crd + L0, p->d_vis + L0,
                                p->d_wgt + L0, p->d_perm + L0, counts.as<int32_t>() + (size_t)b * ntiles, st));
    }
    unsigned long long hb[2];
    IVX_HIP(hipMemcpyAsync(hb, bad.p, sizeof(hb), hipMemcpyDeviceToHost, st));
    IVX_HIP(hipStreamSynchronize(st));
    if (hb[0] != ~0ull || hb[1] != ~0ull) {
        if (hb[0] < hb[1]) return fail(IVX_ENONFINITE, "visibility " + std::to_string(hb[0]) + " is not finite");
        return fail(IVX_EINVAL, "negative weight at visibility " + std::to_string(hb[1]));
    }
    return store_counts(p, counts.as<int32_t>(), ntiles, tstart, st);
}

// Re-sort every block's records for the current tile edge (after a tile change).
ivx_status rebin(ivx_plan *p, hipStream_t st) {
    const Geom &g = p->g;
    const int n_items = g.C * g.P;
    const int ntiles = g.nty * g.ntx;
    int64_t maxn = 0;
    for (int b = 0; b < n_items; ++b) maxn = std::max(maxn, p->block_live[b + 1] - p->block_live[b]);
    const int end_bit = key_bits(ntiles);
    size_t sort_bytes = 0;
    IVX_HIP(sort_pairs(nullptr, sort_bytes, nullptr, nullptr, nullptr, nullptr, (int)std::max<int64_t>(maxn, 1),
                       end_bit, st));
    const bool regeom = p->bin_W != g.W || p->bin_nf != g.nf;
    TmpBuf k1, k2, v1, v2, foot, temp, counts, sc, sv, sw, sp, fr;
    if ((regeom && fr.get(maxn * sizeof(double2)) != hipSuccess) ||
        k1.get(maxn * sizeof(uint64_t)) != hipSuccess || k2.get(maxn * sizeof(uint64_t)) != hipSuccess ||
        v1.get(maxn * sizeof(uint32_t)) != hipSuccess || v2.get(maxn * sizeof(uint32_t)) != hipSuccess ||
        foot.get(maxn * sizeof(int2)) != hipSuccess || temp.get(sort_bytes) != hipSuccess ||
        counts.get((size_t)n_items * ntiles * sizeof(int32_t)) != hipSuccess ||
        sc.get(maxn * sizeof(VisCoord)) != hipSuccess || sv.get(maxn * sizeof(cpx)) != hipSuccess ||
        sw.get(maxn * sizeof(real)) != hipSuccess || sp.get(maxn * sizeof(int32_t)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(IVX_ENOMEM, "device memory for re-binning");
    }
    // every allocation happens before the first record moves: a failure leaves the plan as it was
    int32_t *tstart = nullptr;
    ivx_status s;
    if ((s = dalloc(p, &tstart, (size_t)n_items * (ntiles + 1))) != IVX_OK) return s;
    IVX_HIP(hipMemsetAsync(counts.p, 0, (size_t)n_items * ntiles * sizeof(int32_t), st));
    for (int b = 0; b < n_items; ++b) {
        const int64_t L0 = p->block_live[b], n = p->block_live[b + 1] - L0;
        if (n == 0) continue;
        const Regeom rg{(double)g.nf / (double)p->bin_nf, 0.5 * p->bin_W, 0.5 * g.W, (p->bin_W + 1) / 2, g.O};
        IVX_HIP(launch_rekey(n, p->d_crd + L0, p->d_perm + L0, p->d_tstart + (size_t)b * (p->bin_ntiles + 1),
                             p->bin_ntiles, p->bin_ntx, p->bin_T, g.ntx, g.T, k1.as<uint64_t>(), v1.as<uint32_t>(),
                             foot.as<int2>(), st, regeom ? &rg : nullptr, regeom ? fr.as<double2>() : nullptr));
        size_t tb = sort_bytes;
        IVX_HIP(sort_pairs(temp.p, tb, k1.as<uint64_t>(), k2.as<uint64_t>(), v1.as<uint32_t>(), v2.as<uint32_t>(),
                           (int)n, end_bit, st));
        IVX_HIP(launch_rebin_emit(n, k2.as<uint64_t>(), v2.as<uint32_t>(), foot.as<int2>(), p->d_crd + L0,
                                  p->d_vis + L0, p->d_wgt + L0, p->d_perm + L0, g.ntx, g.T, sc.as<VisCoord>(),
                                  sv.as<cpx>(), sw.as<real>(), sp.as<int32_t>(),
                                  counts.as<int32_t>() + (size_t)b * ntiles, st, regeom ? fr.as<double2>() : nullptr));
        IVX_HIP(hipMemcpyAsync(p->d_crd + L0, sc.p, n * sizeof(VisCoord), hipMemcpyDeviceToDevice, st));
        IVX_HIP(hipMemcpyAsync(p->d_vis + L0, sv.p, n * sizeof(cpx), hipMemcpyDeviceToDevice, st));
        IVX_HIP(hipMemcpyAsync(p->d_wgt + L0, sw.p, n * sizeof(real), hipMemcpyDeviceToDevice, st));
        IVX_HIP(hipMemcpyAsync(p->d_perm + L0, sp.p, n * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    }
    return store_counts(p, counts.as<int32_t>(), ntiles, tstart, st);
}

// Work list (heavy-first), slot map and the tile-dependent buffers, from the record
// counts per (block, tile).
ivx_status build_work(ivx_plan *p, hipStream_t st) {
    Geom &g = p->g;
    const int n_items = g.C * g.P;
    const int ntiles = p->bin_ntiles;
    const int chunk_max = p->chunk_max;
    std::vector<int32_t> tslot((size_t)n_items * (ntiles + 1), 0);
    std::vector<WorkItem> work;
    int64_t slot = 0;
    for (int it = 0; it < n_items; ++it) {
        const int64_t b0 = p->block_live[it];
        const int32_t *cnt = &p->tcount[(size_t)it * ntiles];
        int32_t *ts = &tslot[(size_t)it * (ntiles + 1)];
        int64_t c0 = 0;
        for (int t = 0; t < ntiles; ++t) {
            ts[t] = (int32_t)slot;
            const int64_t c1 = c0 + cnt[t];
            for (int64_t s0 = c0; s0 < c1; s0 += chunk_max) {
                const int64_t c = std::min<int64_t>(chunk_max, c1 - s0);
                WorkItem w;
                w.item = it;
                w.ty = t / g.ntx;
                w.tx = t - (t / g.ntx) * g.ntx;
                w.count = (int32_t)c;
                w.begin = b0 + s0;
                w.slot = (int32_t)slot++;
                w.pad = 0;
                work.push_back(w);
            }
            c0 = c1;
        }
        ts[ntiles] = (int32_t)slot;
        if (slot > INT32_MAX) return fail(IVX_EINVAL, "too many gridding work items: use a larger tile or chunk");
    }
    // heaviest first: blocks are dispatched roughly in index order
    std::stable_sort(work.begin(), work.end(),
                     [](const WorkItem &a, const WorkItem &b) { return a.count > b.count; });
    p->n_work = (int)work.size();
    p->n_slots = (int)slot;
    drop_graph(p); // kernel arguments change with the tiling
    IVX_HIP(prepare_grid(g, p->nwave, p->lanes * 10 + p->vpi));
    for (void *old : {(void *)p->d_work, (void *)p->d_tslot, (void *)p->d_ext, (void *)p->d_slots, (void *)p->d_jpart})
        if (old) free_one(p, old);
    p->d_work = nullptr;
    p->d_tslot = nullptr;
    p->d_ext = p->d_slots = nullptr;
    p->d_jpart = nullptr;
    ivx_status s;
    if ((s = dalloc(p, &p->d_work, std::max<size_t>(work.size(), 1))) != IVX_OK) return s;
    if ((s = dalloc(p, &p->d_tslot, tslot.size())) != IVX_OK) return s;
    if ((s = dalloc(p, &p->d_ext, (size_t)n_items * g.ext_stride)) != IVX_OK) return s;
    if ((s = dalloc(p, &p->d_slots, (size_t)std::max<int64_t>(1, slot) * g.win_stride)) != IVX_OK) return s;
    if ((s = dalloc(p, &p->d_jpart, work.size() + final_scratch((int)work.size()) + 1)) != IVX_OK) return s;
    if (!work.empty())
        IVX_HIP(hipMemcpyAsync(p->d_work, work.data(), work.size() * sizeof(WorkItem), hipMemcpyHostToDevice, st));
    IVX_HIP(hipMemcpyAsync(p->d_tslot, tslot.data(), tslot.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    IVX_HIP(hipStreamSynchronize(st)); // host vectors die at return
    ++p->work_version;
    return IVX_OK;
}

// Tile-dependent device data for the current blocking: records re-sorted when the tile
// edge changed, then the work list.
// A failure leaves the plan without a work list: it needs a successful rebuild (another
// blocking) or set_data before the next evaluation.
ivx_status build_bins(ivx_plan *p, hipStream_t st) {
    ivx_status s = IVX_OK;
    if (p->bin_T != p->g.T || p->bin_W != p->g.W || p->bin_nf != p->g.nf) s = rebin(p, st);
    if (s == IVX_OK) s = build_work(p, st);
    p->has_data = s == IVX_OK;
    return s;
}

ivx_status check_plan(const ivx_plan *p) {
    if (!p) return fail(IVX_EINVAL, "plan is NULL");
    if (!p->has_data) return fail(IVX_ESTATE, "ivx_plan_set_data has not succeeded on this plan");
    return IVX_OK;
}

// check_plan for a call that overwrites the evaluation buffers
ivx_status check_plan_use(ivx_plan *p) {
    ivx_status s = check_plan(p);
    if (s == IVX_OK) ++p->epoch;
    return s;
}

ivx_status run_forward_half(ivx_plan *p, const real *sky, hipStream_t st) {
    const Geom &g = p->g;
    IVX_HIP(launch_image_rows(g, sky, p->d_beams, p->d_interp, p->d_fscale, p->d_dq, p->d_tw, p->d_R, st));
    IVX_HIP(launch_col_fwd(g, p->d_R, p->d_tw, p->d_ext, st));
    return IVX_OK;
}

bool use_fused_fold(const ivx_plan *p) {
    if (!p->fused_fold || !fold_fusable(p->g)) return false;
    return p->fused_fold == 2 || fold_fusion_pays(p->g);
}

// Slots -> inverse column FFT output R: one fused kernel, or the fold into the extended grid
// followed by the column pass.
ivx_status run_fold_col_inv(ivx_plan *p, hipStream_t st) {
    const Geom &g = p->g;
    if (use_fused_fold(p)) {
        IVX_HIP(launch_col_inv_slots(g, p->d_tslot, p->d_slots, p->d_tw, p->d_R, st));
    } else {
        IVX_HIP(launch_fold(g, p->d_tslot, p->d_slots, p->d_ext, st));
        IVX_HIP(launch_col_inv(g, p->d_ext, p->d_tw, p->d_R, st));
    }
    return IVX_OK;
}

ivx_status run_adjoint_half(ivx_plan *p, hipStream_t st) {
    const Geom &g = p->g;
    ivx_status s = run_fold_col_inv(p, st);
    if (s != IVX_OK) return s;
    IVX_HIP(launch_row_inv(g, p->d_R, p->d_beams, p->d_fscale, p->d_dq, p->d_tw, p->d_gp, st));
    return IVX_OK;
}

bool sd_active(const ivx_plan *p) { return p->d.lambda_s != 0.0 && p->d.sd_n > 0; }

// weight of the spectral term as the sky pass sees it (0 when it is off or there is one channel)
real spec_weight(const ivx_plan *p) { return p->g.C > 1 ? (real)p->d.lambda_nu : real(0); }

// Event pair around one stage when timing is on (start before the launch, stop after).
hipEvent_t next_event(ivx_plan *p) {
    if (p->ev_next == p->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        p->ev_pool.push_back(e);
    }
    return p->ev_pool[p->ev_next++];
}

struct StageTimer {
    ivx_plan *p;
    hipStream_t st;
    int stage;
    hipEvent_t stop = nullptr;
    StageTimer(ivx_plan *p_, hipStream_t st_, int stage_) : p(p_), st(st_), stage(stage_) {
        if (!(p->timing_mask & (1u << stage))) return;
        const size_t i0 = p->ev_next;
        hipEvent_t start = next_event(p);
        stop = next_event(p);
        if (!start || !stop || hipEventRecord(start, st) != hipSuccess) {
            stop = nullptr;
            return;
        }
        p->ev_used.push_back({stage, (int)i0});
    }
    ~StageTimer() {
        if (stop) (void)hipEventRecord(stop, st);
    }
};

ivx_status eval_objective(ivx_plan *p, const real *sky, real *grad, double *terms_dev, hipStream_t st) {
    const Geom &g = p->g;
    if (p->timing_mask) p->timed_evals++;
    {
        StageTimer t(p, st, IVX_STAGE_IMAGE_ROWS);
        IVX_HIP(launch_image_rows(g, sky, p->d_beams, p->d_interp, p->d_fscale, p->d_dq, p->d_tw, p->d_R, st));
    }
    {
        StageTimer t(p, st, IVX_STAGE_COL_FWD);
        IVX_HIP(launch_col_fwd(g, p->d_R, p->d_tw, p->d_ext, st));
    }
    {
        StageTimer t(p, st, IVX_STAGE_GRID);
        IVX_HIP(launch_grid(MODE_OBJ, g, p->d_work, p->n_work, p->d_crd, p->d_vis, p->d_wgt, p->d_perm, p->d_boff, p->d_ext,
                            p->d_slots, p->d_jpart, nullptr, nullptr, p->nwave, p->lanes * 10 + p->vpi, p->occupancy, st));
    }
    if (use_fused_fold(p)) {
        StageTimer t(p, st, IVX_STAGE_COL_INV); // the fold happens inside this stage
        IVX_HIP(launch_col_inv_slots(g, p->d_tslot, p->d_slots, p->d_tw, p->d_R, st));
    } else {
        {
            StageTimer t(p, st, IVX_STAGE_FOLD);
            IVX_HIP(launch_fold(g, p->d_tslot, p->d_slots, p->d_ext, st));
        }
        StageTimer t(p, st, IVX_STAGE_COL_INV);
        IVX_HIP(launch_col_inv(g, p->d_ext, p->d_tw, p->d_R, st));
    }
    {
        StageTimer t(p, st, IVX_STAGE_ROW_INV);
        IVX_HIP(launch_row_inv(g, p->d_R, p->d_beams, p->d_fscale, p->d_dq, p->d_tw, p->d_gp, st));
    }
    const bool sd = sd_active(p);
    if (sd) {
        StageTimer t(p, st, IVX_STAGE_SD);
        IVX_HIP(launch_sd_rows(g, sky, p->d_gB, p->sd_rb, p->d.sd_n, p->d.sd_stride, p->d.sd_offset, p->d_U, st));
        IVX_HIP(launch_sd_cols(g, p->d_U, p->d_gB, p->sd_rb, p->d.sd_n, p->d.sd_stride, p->d.sd_offset, p->d_sdmap,
                               (real)(1.0 / (p->d.sd_sigma * p->d.sd_sigma)), p->d_E, p->d_kpart, st));
        // U is free again: it receives the column half of the adjoint for the sky pass
        IVX_HIP(launch_sd_back(g, p->d_E, p->d_gB, p->sd_rb, p->d.sd_n, p->d.sd_stride, p->d.sd_offset, p->d_U, st));
    }
    {
        StageTimer t(p, st, IVX_STAGE_SKY);
        IVX_HIP(launch_sky(g, sky, p->d_gp, p->d_cptr, p->d_cent, (real)p->d.lambda_r,
                           sd ? (real)p->d.lambda_s : real(0), p->d_U, p->d_gB, p->sd_rb, p->d.sd_n, p->d.sd_stride,
                           p->d.sd_offset, grad, p->d_rpart, SKY_FULL, real(1), st, spec_weight(p), p->d_npart));
    }
    {
        StageTimer t(p, st, IVX_STAGE_FINAL);
        IVX_HIP(launch_final(p->d_jpart, p->n_work, p->d_jpart + p->n_work, p->d_rpart, p->n_rpart, p->d_kpart,
                             sd ? p->n_kpart : 0, p->d_npart, spec_weight(p) != real(0) ? p->n_rpart : 0,
                             p->d.lambda_r, sd ? p->d.lambda_s : 0.0, p->d.lambda_nu, p->d_terms, terms_dev, st));
    }
    return IVX_OK;
}

// Forward half of an evaluation: the visibility model, residual and data term (MODE_OBJ also
// spreads the weighted residual into the slots for a following adjoint half, MODE_VAL does
// not), the single-dish model and residual, the regulariser value, and the four totals.
ivx_status eval_value(ivx_plan *p, const real *sky, double *terms_dev, int grid_mode, hipStream_t st) {
    const Geom &g = p->g;
    IVX_HIP(launch_image_rows(g, sky, p->d_beams, p->d_interp, p->d_fscale, p->d_dq, p->d_tw, p->d_R, st));
    IVX_HIP(launch_col_fwd(g, p->d_R, p->d_tw, p->d_ext, st));
    IVX_HIP(launch_grid(grid_mode, g, p->d_work, p->n_work, p->d_crd, p->d_vis, p->d_wgt, p->d_perm, p->d_boff,
                        p->d_ext, p->d_slots, p->d_jpart, nullptr, nullptr, p->nwave, p->lanes * 10 + p->vpi,
                        p->occupancy, st));
    const bool sd = sd_active(p);
    if (sd) {
        IVX_HIP(launch_sd_rows(g, sky, p->d_gB, p->sd_rb, p->d.sd_n, p->d.sd_stride, p->d.sd_offset, p->d_U, st));
        IVX_HIP(launch_sd_cols(g, p->d_U, p->d_gB, p->sd_rb, p->d.sd_n, p->d.sd_stride, p->d.sd_offset, p->d_sdmap,
                               (real)(1.0 / (p->d.sd_sigma * p->d.sd_sigma)), p->d_E, p->d_kpart, st));
        if (grid_mode == MODE_OBJ)
            IVX_HIP(launch_sd_back(g, p->d_E, p->d_gB, p->sd_rb, p->d.sd_n, p->d.sd_stride, p->d.sd_offset, p->d_U, st));
    }
    IVX_HIP(launch_sky(g, sky, p->d_gp, p->d_cptr, p->d_cent, (real)p->d.lambda_r, real(0), nullptr, nullptr, 0, 0, 1,
                       0, nullptr, p->d_rpart, SKY_VALUE, real(1), st, spec_weight(p), p->d_npart));
    IVX_HIP(launch_final(p->d_jpart, p->n_work, p->d_jpart + p->n_work, p->d_rpart, p->n_rpart, p->d_kpart,
                         sd ? p->n_kpart : 0, p->d_npart, spec_weight(p) != real(0) ? p->n_rpart : 0, p->d.lambda_r,
                         sd ? p->d.lambda_s : 0.0, p->d.lambda_nu, p->d_terms, terms_dev, st));
    return IVX_OK;
}

// Adjoint half after eval_value(MODE_OBJ): slots -> inverse FFTs -> reprojection transpose,
// plus the regulariser and single-dish gradients, all multiplied by `scale`.
ivx_status eval_gradient(ivx_plan *p, const real *sky, real *grad, real scale, hipStream_t st) {
    const Geom &g = p->g;
    ivx_status s = run_adjoint_half(p, st);
    if (s != IVX_OK) return s;
    const bool sd = sd_active(p);
    IVX_HIP(launch_sky(g, sky, p->d_gp, p->d_cptr, p->d_cent, (real)p->d.lambda_r, sd ? (real)p->d.lambda_s : real(0),
                       p->d_U, p->d_gB, p->sd_rb, p->d.sd_n, p->d.sd_stride, p->d.sd_offset, grad, p->d_rpart,
                       SKY_FULL, scale, st, spec_weight(p), p->d_npart));
    return IVX_OK;
}

// ---------------------------------------------------------------- full forward model
// The w kernel (W_w planes, oversampling sigma_w) and the per-pixel tables of the sub-image:
// x' = (n - 1) - x_c, dw x', and 1 / (n Phi(dw x')).  Fails if a pixel lies outside the unit
// circle of direction cosines.
ivx_status w_tables(ivx_plan *p, int Ww, double sigma) {
    const Geom &g = p->g;
    const int nk = g.nk, c = nk / 2;
    const double delta = p->d.pixel_rad;
    const int64_t nk2 = (int64_t)nk * nk;
    std::vector<double> nm1(nk2), nn(nk2);
    double xmin = 0.0;
    for (int a = 0; a < nk; ++a)
        for (int b = 0; b < nk; ++b) {
            const double l = (b - c) * delta, m = (a - c) * delta, r2 = l * l + m * m;
            if (!(r2 < 1.0)) return fail(IVX_EINVAL, "a sub-image pixel lies outside the unit circle of direction cosines");
            const double n = std::sqrt(1.0 - r2);
            nn[(size_t)a * nk + b] = n;
            nm1[(size_t)a * nk + b] = -r2 / (1.0 + n);
            xmin = std::min(xmin, nm1[(size_t)a * nk + b]);
        }
    if (!(xmin < 0.0)) return fail(IVX_EINVAL, "the sub-image has no extent in n - 1");
    p->w_W = Ww;
    p->w_sigma = sigma;
    p->w_beta = 2.30 * Ww * (1.0 - 1.0 / (2.0 * sigma)) / 0.75;
    p->w_xc = 0.5 * xmin;
    p->w_X = -xmin;
    p->w_dw = 1.0 / (sigma * p->w_X);
    std::vector<double> gx, gw, xp(nk2), tp(nk2);
    std::vector<real> corr(nk2);
    gauss_legendre(std::max(64, 8 * Ww), gx, gw);
    for (int64_t i = 0; i < nk2; ++i) {
        xp[i] = nm1[i] - p->w_xc;
        tp[i] = p->w_dw * xp[i];
        corr[i] = (real)(1.0 / (nn[i] * es_phihat(2.0 * M_PI * tp[i], Ww, p->w_beta, gx, gw)));
    }
    ivx_status s;
    if (!p->d_wxp) {
        if ((s = dalloc(p, &p->d_wxp, nk2)) != IVX_OK || (s = dalloc(p, &p->d_wtp, nk2)) != IVX_OK ||
            (s = dalloc(p, &p->d_wcorr, nk2)) != IVX_OK)
            return s;
    }
    IVX_HIP(hipMemcpy(p->d_wxp, xp.data(), nk2 * sizeof(double), hipMemcpyHostToDevice));
    IVX_HIP(hipMemcpy(p->d_wtp, tp.data(), nk2 * sizeof(double), hipMemcpyHostToDevice));
    IVX_HIP(hipMemcpy(p->d_wcorr, corr.data(), nk2 * sizeof(real), hipMemcpyHostToDevice));
    return IVX_OK;
}

// The caller's w of block b (device copy) and its scale.
const real *w_source(const ivx_plan *p, int b, double &scale) {
    const int k = b / p->g.C, c = b - (b / p->g.C) * p->g.C;
    if (p->shared_uv) {
        scale = p->uv_scale[c];
        return p->d_wsrc + p->pt_off[k];
    }
    scale = 1.0;
    return p->d_wsrc + p->offsets[b];
}

// Plane coordinates of the records for the current work list: per-block w range and plane
// count, zeta of every record, and the records of each work item sorted by zeta.  Runs when
// the work list changed since the last preparation.
ivx_status w_prepare(ivx_plan *p, hipStream_t st) {
    if (!p->w_on || p->w_version == p->work_version) return IVX_OK;
    const Geom &g = p->g;
    const int n_items = g.C * g.P;
    if (p->chunk_max > WSORT_MAX)
        return fail(IVX_EINVAL, "the full model needs work items of at most " + std::to_string(WSORT_MAX) +
                                    " visibilities: set a smaller chunk with ivx_set_blocking");
    const int wrb = wrange_blocks();
    TmpBuf part, bad;
    IVX_HIP(part.get((size_t)n_items * wrb * 2 * sizeof(double)));
    IVX_HIP(bad.get(sizeof(unsigned int)));
    double *pmin = part.as<double>(), *pmax = pmin + (size_t)n_items * wrb;
    for (int b = 0; b < n_items; ++b) {
        const int64_t L0 = p->block_live[b], n = p->block_live[b + 1] - L0;
        double scale;
        const real *ws = w_source(p, b, scale);
        IVX_HIP(launch_wrange(n, p->d_perm + L0, ws, scale, pmin + (size_t)b * wrb, pmax + (size_t)b * wrb, st));
    }
    std::vector<double> hp((size_t)n_items * wrb * 2);
    IVX_HIP(hipMemcpyAsync(hp.data(), part.p, hp.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    IVX_HIP(hipStreamSynchronize(st));
    p->w0_host.assign(n_items, 0.0);
    p->np_host.assign(n_items, 0);
    int planes = 0;
    const double dw = p->w_dw;
    const int W = p->w_W;
    for (int b = 0; b < n_items; ++b) {
        if (p->block_live[b + 1] == p->block_live[b]) continue;
        double lo = INFINITY, hi = -INFINITY;
        for (int i = 0; i < wrb; ++i) {
            lo = std::min(lo, hp[(size_t)b * wrb + i]);
            hi = std::max(hi, hp[(size_t)n_items * wrb + (size_t)b * wrb + i]);
        }
        if (!std::isfinite(lo) || !std::isfinite(hi)) return fail(IVX_ENONFINITE, "w holds a non-finite value");
        const double span = (hi - lo) / dw;
        const double np = std::floor(span - 0.5) + W + 1;
        if (np > (double)WZ_MAX_PLANES)
            return fail(IVX_EINVAL, "block " + std::to_string(b) + " spans " + std::to_string((int64_t)np) +
                                        " w planes (at most " + std::to_string(WZ_MAX_PLANES) +
                                        "): lower w_sigma or the sub-image extent");
        p->np_host[b] = (int32_t)np;
        p->w0_host[b] = lo - dw * 0.5 * (W - 1);
        planes = std::max(planes, (int)np);
    }
    ivx_status s;
    if (!p->d_w0) {
        if ((s = dalloc(p, &p->d_w0, n_items)) != IVX_OK || (s = dalloc(p, &p->d_wnp, n_items)) != IVX_OK) return s;
    }
    if (!p->d_wz) {
        const size_t L = (size_t)std::max<int64_t>(p->m_live, 1);
        if ((s = dalloc(p, &p->d_wz, L)) != IVX_OK || (s = dalloc(p, &p->d_wacc, L)) != IVX_OK) return s;
    }
    if (p->n_slots != p->wsact_count) {
        if (p->d_wsact) free_one(p, p->d_wsact);
        p->d_wsact = nullptr;
        p->wsact_count = 0;
        if ((s = dalloc(p, &p->d_wsact, (size_t)std::max(p->n_slots, 1))) != IVX_OK) return s;
        p->wsact_count = p->n_slots;
    }
    const size_t wr = (size_t)n_items * g.nk * g.ew;
    if (wr != p->wR_count) {
        if (p->d_wR) free_one(p, p->d_wR);
        p->d_wR = nullptr;
        p->wR_count = 0;
        if ((s = dalloc(p, &p->d_wR, wr)) != IVX_OK) return s;
        p->wR_count = wr;
    }
    IVX_HIP(hipMemcpyAsync(p->d_w0, p->w0_host.data(), n_items * sizeof(double), hipMemcpyHostToDevice, st));
    IVX_HIP(hipMemcpyAsync(p->d_wnp, p->np_host.data(), n_items * sizeof(int32_t), hipMemcpyHostToDevice, st));
    IVX_HIP(hipMemsetAsync(bad.p, 0, sizeof(unsigned int), st));
    for (int b = 0; b < n_items; ++b) {
        const int64_t L0 = p->block_live[b], n = p->block_live[b + 1] - L0;
        double scale;
        const real *ws = w_source(p, b, scale);
        IVX_HIP(launch_wzeta(n, p->d_perm + L0, ws, scale, p->w0_host[b], 1.0 / dw, p->d_wz + L0, bad.as<unsigned int>(),
                             st));
    }
    IVX_HIP(launch_wsort(p->d_work, p->n_work, p->d_crd, p->d_vis, p->d_wgt, p->d_perm, p->d_wz, st));
    // the plane ranges of every work item as a table (two loads per work item and plane in the
    // gridding passes instead of two binary searches), when it fits a modest budget
    if (p->d_wcnt) free_one(p, p->d_wcnt);
    p->d_wcnt = nullptr;
    p->wncnt = 0;
    {
        const int ncnt = 2 * planes + W + 1;
        const size_t bytes = (size_t)std::max(p->n_work, 1) * ncnt * sizeof(int32_t);
        if (planes > 0 && bytes <= ((size_t)2 << 30) && dalloc(p, &p->d_wcnt, bytes / sizeof(int32_t)) == IVX_OK) {
            p->wncnt = ncnt;
            IVX_HIP(launch_wcounts(p->d_work, p->n_work, p->d_wz, ncnt, p->d_wcnt, st));
        } else {
            g_last_error.clear(); // the binary searches serve instead
        }
    }
    IVX_HIP(prepare_wgrid(g, p->nwave));
    unsigned int hb = 0;
    IVX_HIP(hipMemcpyAsync(&hb, bad.p, sizeof(hb), hipMemcpyDeviceToHost, st));
    IVX_HIP(hipStreamSynchronize(st)); // host vectors die at return
    if (hb) return fail(IVX_ENONFINITE, "a w value is not finite");
    p->w_planes = planes;
    p->w_version = p->work_version;
    return IVX_OK;
}

WGeom wgeom(const ivx_plan *p) {
    const Geom &g = p->g;
    return WGeom{p->d_wnp, p->d_w0, p->d_wxp, p->d_wtp, p->d_wcorr, p->w_dw, p->w_xc, std::min(g.ew, g.nf),
                 (int64_t)g.nk * g.ew};
}

WPlane wplane(const ivx_plan *p, int plane, bool adjoint) {
    return WPlane{p->d_wz, adjoint ? nullptr : p->d_wacc, adjoint ? p->d_wacc : nullptr, plane, p->w_W, p->w_beta,
                  p->d_wcnt, p->wncnt, adjoint ? p->d_wsact : nullptr};
}

// Sky -> per-record sum over planes of the w-kernel-weighted plane transforms (d_wacc).
ivx_status w_forward_planes(ivx_plan *p, const real *sky, hipStream_t st) {
    const Geom &g = p->g;
    const WGeom wg = wgeom(p);
    IVX_HIP(launch_zero(p->d_wacc, std::max<int64_t>(p->m_live, 1) * (int64_t)sizeof(cpx), st));
    for (int pl = 0; pl < p->w_planes; ++pl) {
        {
            StageTimer t(p, st, IVX_STAGE_IMAGE_ROWS);
            IVX_HIP(launch_wplane_rows(g, wg, pl, sky, p->d_beams, p->d_interp, p->d_fscale, p->d_dq, p->d_tw,
                                       p->d_wR, st));
        }
        {
            StageTimer t(p, st, IVX_STAGE_COL_FWD);
            IVX_HIP(launch_wplane_cols(g, wg, pl, p->d_wR, p->d_tw, p->d_ext, st));
        }
        StageTimer t(p, st, IVX_STAGE_GRID);
        IVX_HIP(launch_wgrid(MODE_WFWD, g, p->d_work, p->n_work, p->d_crd, p->d_ext, p->d_slots, wplane(p, pl, false),
                             p->nwave, p->lanes * 10 + p->vpi, p->occupancy, st));
    }
    return IVX_OK;
}

// Per-record adjoint coefficients (d_wacc) -> image gradient of every block (d_gp).
ivx_status w_adjoint_planes(ivx_plan *p, hipStream_t st) {
    const Geom &g = p->g;
    const WGeom wg = wgeom(p);
    if (p->w_planes == 0)
        IVX_HIP(launch_zero(p->d_gp, (int64_t)g.C * g.P * g.nk * g.nk * (int64_t)sizeof(real), st));
    for (int pl = 0; pl < p->w_planes; ++pl) {
        {
            StageTimer t(p, st, IVX_STAGE_GRID);
            IVX_HIP(launch_wgrid(MODE_WADJ, g, p->d_work, p->n_work, p->d_crd, p->d_ext, p->d_slots,
                                 wplane(p, pl, true), p->nwave, p->lanes * 10 + p->vpi, p->occupancy, st));
        }
        {
            StageTimer t(p, st, IVX_STAGE_FOLD);
            IVX_HIP(launch_fold(g, p->d_tslot, p->d_slots, p->d_ext, st, p->d_wsact));
        }
        {
            StageTimer t(p, st, IVX_STAGE_COL_INV);
            IVX_HIP(launch_wplane_cols_inv(g, wg, pl, p->d_ext, p->d_tw, p->d_wR, st));
        }
        StageTimer t(p, st, IVX_STAGE_ROW_INV);
        IVX_HIP(launch_wplane_rows_inv(g, wg, pl, p->d_wR, p->d_beams, p->d_fscale, p->d_dq, p->d_tw, p->d_gp, st));
    }
    return IVX_OK;
}

// eval_value / eval_gradient of the full model.
ivx_status eval_value_w(ivx_plan *p, const real *sky, double *terms_dev, bool keep_sd_adjoint, hipStream_t st) {
    const Geom &g = p->g;
    if (p->timing_mask) p->timed_evals++;
    ivx_status s = w_forward_planes(p, sky, st);
    if (s != IVX_OK) return s;
    {
        StageTimer t(p, st, IVX_STAGE_GRID);
        IVX_HIP(launch_wresid(p->d_work, p->n_work, wgeom(p), p->d_wz, p->d_vis, p->d_wgt, p->d_wacc, p->d_jpart, st));
    }
    const bool sd = sd_active(p);
    if (sd) {
        StageTimer t(p, st, IVX_STAGE_SD);
        IVX_HIP(launch_sd_rows(g, sky, p->d_gB, p->sd_rb, p->d.sd_n, p->d.sd_stride, p->d.sd_offset, p->d_U, st));
        IVX_HIP(launch_sd_cols(g, p->d_U, p->d_gB, p->sd_rb, p->d.sd_n, p->d.sd_stride, p->d.sd_offset, p->d_sdmap,
                               (real)(1.0 / (p->d.sd_sigma * p->d.sd_sigma)), p->d_E, p->d_kpart, st));
        if (keep_sd_adjoint)
            IVX_HIP(launch_sd_back(g, p->d_E, p->d_gB, p->sd_rb, p->d.sd_n, p->d.sd_stride, p->d.sd_offset, p->d_U, st));
    }
    IVX_HIP(launch_sky(g, sky, p->d_gp, p->d_cptr, p->d_cent, (real)p->d.lambda_r, real(0), nullptr, nullptr, 0, 0, 1,
                       0, nullptr, p->d_rpart, SKY_VALUE, real(1), st, spec_weight(p), p->d_npart));
    IVX_HIP(launch_final(p->d_jpart, p->n_work, p->d_jpart + p->n_work, p->d_rpart, p->n_rpart, p->d_kpart,
                         sd ? p->n_kpart : 0, p->d_npart, spec_weight(p) != real(0) ? p->n_rpart : 0, p->d.lambda_r,
                         sd ? p->d.lambda_s : 0.0, p->d.lambda_nu, p->d_terms, terms_dev, st));
    return IVX_OK;
}

ivx_status eval_gradient_w(ivx_plan *p, const real *sky, real *grad, real scale, hipStream_t st) {
    const Geom &g = p->g;
    ivx_status s = w_adjoint_planes(p, st);
    if (s != IVX_OK) return s;
    const bool sd = sd_active(p);
    StageTimer t(p, st, IVX_STAGE_SKY);
    IVX_HIP(launch_sky(g, sky, p->d_gp, p->d_cptr, p->d_cent, (real)p->d.lambda_r, sd ? (real)p->d.lambda_s : real(0),
                       p->d_U, p->d_gB, p->sd_rb, p->d.sd_n, p->d.sd_stride, p->d.sd_offset, grad, p->d_rpart,
                       SKY_FULL, scale, st, spec_weight(p), p->d_npart));
    return IVX_OK;
}

// ivx_adjoint / ivx_forward_adjoint of the full model: caller coefficients (times the natural
// weights unless `unweighted`) -> planes -> reprojection transpose into `image`.
ivx_status w_adjoint_call(ivx_plan *p, const real *vis, real *image, bool unweighted, hipStream_t st) {
    ivx_status s = w_prepare(p, st);
    if (s != IVX_OK) return s;
    IVX_HIP(launch_win(p->d_work, p->n_work, wgeom(p), p->d_wz, p->d_perm, p->d_boff, p->d_wgt, unweighted,
                       reinterpret_cast<const cpx *>(vis), p->d_wacc, st));
    if ((s = w_adjoint_planes(p, st)) != IVX_OK) return s;
    IVX_HIP(launch_sky(p->g, image, p->d_gp, p->d_cptr, p->d_cent, real(0), real(0), nullptr, nullptr, 0, 0, 1, 0,
                       image, p->d_rpart, SKY_ADJOINT, real(1), st));
    return IVX_OK;
}

// Device pointer for `terms` (written by the last kernel) or nullptr for host memory.
double *device_terms(double *terms) {
    if (!terms) return nullptr;
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, terms) == hipSuccess) {
        if (attr.type == hipMemoryTypeDevice) return terms;
    } else {
        (void)hipGetLastError();
    }
    return nullptr;
}

ivx_status copy_terms(ivx_plan *p, double *terms, double *terms_dev, hipStream_t st) {
    if (terms && !terms_dev) {
        IVX_HIP(hipMemcpyAsync(terms, p->d_terms, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
        IVX_HIP(hipStreamSynchronize(st));
    }
    return IVX_OK;
}

} // namespace

// ====================================================================== C ABI

namespace {
ivx_status set_data_impl(ivx_plan *p, const VisSource &src, bool shared, const ivx_real *beams,
                         const ivx_real *interp, const ivx_real *sd_map, void *stream);
} // namespace

namespace ivx {
// Number of sky variables of a plan (n_chan * n_sky^2), for the bounded solver.
int64_t plan_sky_count(const ivx_plan *p) { return p ? (int64_t)p->g.C * p->g.N * p->g.N : 0; }
} // namespace ivx

extern "C" {

const char *ivx_last_error(void) { return g_last_error.c_str(); }

int ivx_version(void) { return IVX_VERSION; }

int ivx_real_size(void) { return (int)sizeof(ivx_real); }

ivx_status ivx_plan_create(const ivx_problem *d, ivx_plan **out) {
    g_last_error.clear();
    if (!out) return fail(IVX_EINVAL, "out is NULL");
    *out = nullptr;
    if (!d) return fail(IVX_EINVAL, "problem is NULL");
    if (d->n_chan < 1 || d->n_point < 1) return fail(IVX_EINVAL, "n_chan and n_point must be >= 1");
    if (d->n_sky < 4 || d->n_sky > 65536) return fail(IVX_EINVAL, "n_sky must be in [4, 65536]");
    if (d->n_sub < 4 || (d->n_sub & 1) || d->n_sub > 1024) return fail(IVX_EINVAL, "n_sub must be even in [4, 1024]");
    if (!(d->pixel_rad > 0.0) || !std::isfinite(d->pixel_rad)) return fail(IVX_EINVAL, "pixel_rad must be > 0");
    if (!d->vis_offsets || !d->flux_scale) return fail(IVX_EINVAL, "vis_offsets and flux_scale are required");
    if (!(d->lambda_r >= 0.0) || !(d->lambda_s >= 0.0) || !std::isfinite(d->lambda_r) || !std::isfinite(d->lambda_s))
        return fail(IVX_EINVAL, "lambda_r and lambda_s must be finite and >= 0");
    if (!(d->lambda_nu >= 0.0) || !std::isfinite(d->lambda_nu)) return fail(IVX_EINVAL, "lambda_nu must be finite and >= 0");
    if (d->reserved != 0) return fail(IVX_EINVAL, "reserved must be 0");
    const int64_t nb = (int64_t)d->n_point * d->n_chan;
    if (nb > (1 << 24)) return fail(IVX_EINVAL, "too many (pointing, channel) blocks");
    if (d->vis_offsets[0] != 0) return fail(IVX_EINVAL, "vis_offsets[0] must be 0");
    for (int64_t i = 0; i < nb; ++i)
        if (d->vis_offsets[i + 1] < d->vis_offsets[i]) return fail(IVX_EINVAL, "vis_offsets must be non-decreasing");
    for (int c = 0; c < d->n_chan; ++c)
        if (!std::isfinite(d->flux_scale[c])) return fail(IVX_EINVAL, "flux_scale must be finite");
    if (d->sd_n < 0) return fail(IVX_EINVAL, "sd_n must be >= 0");
    if (d->sd_n > 0) {
        if (d->sd_stride < 1 || d->sd_offset < 0 || d->sd_offset + (int64_t)(d->sd_n - 1) * d->sd_stride >= d->n_sky)
            return fail(IVX_EINVAL, "single-dish samples must lie inside the sky");
        if (!(d->sd_fwhm_rad > 0.0) || !(d->sd_sigma > 0.0)) return fail(IVX_EINVAL, "sd_fwhm_rad and sd_sigma must be > 0");
    }
    ivx_plan *p = new (std::nothrow) ivx_plan();
    if (!p) return fail(IVX_ENOMEM, "host allocation of the plan failed");
    p->d = *d;
    p->offsets.assign(d->vis_offsets, d->vis_offsets + nb + 1);
    p->fscale.assign(d->flux_scale, d->flux_scale + d->n_chan);
    p->d.vis_offsets = nullptr;
    p->d.flux_scale = nullptr;
    p->m_total = p->offsets.back();

    Geom &g = p->g;
    g.C = d->n_chan;
    g.P = d->n_point;
    g.N = d->n_sky;
    g.nk = d->n_sub;
    int nf = d->fine_size;
    if (nf == 0) {
        nf = 64;
        while (nf < 2 * d->n_sub) nf *= 2;
    }
    if (!is_pow2(nf) || nf < 64 || nf > 2048 || nf * 4 < d->n_sub * 5) {
        delete p;
        return fail(IVX_EINVAL, "fine_size must be a power of two in [64, 2048] and >= 1.25 n_sub");
    }
    const double sigma = (double)nf / d->n_sub;
    int W = d->kernel_width;
    if (W == 0) {
        double eps = d->nufft_eps;
        if (eps <= 0.0) eps = sizeof(real) == 4 ? 1e-7 : 1e-12;
        W = (int)std::ceil(std::log(1.0 / eps) / (M_PI * std::sqrt(1.0 - 1.0 / sigma)));
        W = std::max(4, std::min(16, W));
    }
    if (W < 4 || W > 16) {
        delete p;
        return fail(IVX_EINVAL, "kernel_width must be in [4, 16]");
    }
    set_geometry_fields(p, W, nf);
    p->geometry_auto = d->kernel_width == 0 && d->fine_size == 0;
    p->eps_target = d->nufft_eps > 0.0 ? d->nufft_eps : nufft_probe_error(g.nk, nf, W);
    p->tile_fixed = d->tile;
    bool ok = false;
    if (d->tile == 0) {
        ok = auto_blocking(p);
    } else {
        for (int nw : {4, 2, 1})
            if (tile_fits(p, d->tile, nw, 16)) {
                p->nwave = nw;
                set_tile(p, d->tile);
                ok = true;
                break;
            }
    }
    if (!ok) {
        delete p;
        return fail(IVX_EINVAL, "tile must be >= kernel_width and fit the LDS");
    }
    if (d->sd_n > 0) {
        const double sig = d->sd_fwhm_rad / (2.0 * std::sqrt(2.0 * std::log(2.0)));
        p->sd_rb = (int)std::ceil(4.0 * sig / d->pixel_rad);
        std::vector<double> taps(2 * p->sd_rb + 1);
        double sum = 0.0;
        for (int t = -p->sd_rb; t <= p->sd_rb; ++t) {
            const double v = std::exp(-(t * d->pixel_rad) * (t * d->pixel_rad) / (2.0 * sig * sig));
            taps[t + p->sd_rb] = v;
            sum += v;
        }
        p->gB_host.resize(taps.size());
        for (size_t i = 0; i < taps.size(); ++i) p->gB_host[i] = (real)(taps[i] / sum);
    }
    *out = p;
    return IVX_OK;
}

ivx_status ivx_set_blocking(ivx_plan *p, int32_t tile, int32_t waves, int32_t chunk, int32_t lanes, int32_t vpi,
                            void *stream) {
    if (!p) return fail(IVX_EINVAL, "plan is NULL");
    if (!(waves == 1 || waves == 2 || waves == 4) || chunk < 16 ||
        !(lanes == 8 || lanes == 16 || lanes == GRID_MFMA_LANES) || !(vpi == 1 || vpi == 2) ||
        (lanes == GRID_MFMA_LANES && vpi != 1))
        return fail(IVX_EINVAL, "blocking out of range");
    if (!tile_fits(p, tile, waves, lanes)) return fail(IVX_EINVAL, "blocking does not fit the LDS");
    ++p->epoch;
    p->nwave = waves;
    p->chunk_max = chunk;
    p->lanes = lanes;
    p->vpi = vpi;
    set_tile(p, tile);
    if (p->bin_T > 0) { // records exist (set_data succeeded)
        ivx_status s = build_bins(p, (hipStream_t)stream);
        if (s != IVX_OK) return s;
    }
    return IVX_OK;
}

ivx_status ivx_set_gridder_occupancy(ivx_plan *p, int32_t waves_per_simd) {
    if (!p) return fail(IVX_EINVAL, "plan is NULL");
    if (!(waves_per_simd == 0 || waves_per_simd == 6 || waves_per_simd == 7))
        return fail(IVX_EINVAL, "waves_per_simd must be 0 (automatic), 6 or 7");
    p->occupancy = waves_per_simd;
    drop_graph(p); // the captured launches name the build
    return IVX_OK;
}

ivx_status ivx_set_fused_fold(ivx_plan *p, int enable) {
    if (!p) return fail(IVX_EINVAL, "plan is NULL");
    if (enable < 0 || enable > 2) return fail(IVX_EINVAL, "enable must be 0, 1 or 2");
    p->fused_fold = enable;
    drop_graph(p);
    return IVX_OK;
}

ivx_status ivx_set_graph(ivx_plan *p, int enable) {
    if (!p) return fail(IVX_EINVAL, "plan is NULL");
    p->use_graph = enable != 0;
    if (!p->use_graph) drop_graph(p);
    return IVX_OK;
}

ivx_status ivx_set_timing(ivx_plan *p, uint32_t stage_mask) {
    if (!p) return fail(IVX_EINVAL, "plan is NULL");
    p->timing_mask = stage_mask & ((1u << IVX_NSTAGE) - 1u);
    return IVX_OK;
}

ivx_status ivx_stage_times(ivx_plan *p, double *ms, int64_t *n_eval) {
    if (!p || !ms) return fail(IVX_EINVAL, "plan and ms must be non-NULL");
    for (int i = 0; i < IVX_NSTAGE; ++i) ms[i] = 0.0;
    for (const auto &u : p->ev_used) {
        hipEvent_t a = p->ev_pool[u.second], b = p->ev_pool[u.second + 1];
        IVX_HIP(hipEventSynchronize(b));
        float t = 0.f;
        IVX_HIP(hipEventElapsedTime(&t, a, b));
        ms[u.first] += t;
    }
    if (n_eval) *n_eval = p->timed_evals;
    p->ev_used.clear();
    p->ev_next = 0;
    p->timed_evals = 0;
    return IVX_OK;
}

ivx_status ivx_last_terms(ivx_plan *p, double *terms5, void *stream) {
    ivx_status s = check_plan(p);
    if (s != IVX_OK) return s;
    if (!terms5) return fail(IVX_EINVAL, "terms5 is required");
    hipStream_t st = (hipStream_t)stream;
    IVX_HIP(hipMemcpyAsync(terms5, p->d_terms, 5 * sizeof(double), hipMemcpyDeviceToHost, st));
    IVX_HIP(hipStreamSynchronize(st));
    return IVX_OK;
}

ivx_status ivx_plan_destroy(ivx_plan *plan) {
    if (!plan) return IVX_OK;
    for (hipEvent_t e : plan->ev_pool) (void)hipEventDestroy(e);
    plan->ev_pool.clear();
    free_all(plan);
    if (plan->cap_stream) (void)hipStreamDestroy(plan->cap_stream);
    delete plan;
    return IVX_OK;
}

ivx_status ivx_plan_info(const ivx_plan *p, int64_t *info) {
    if (!p || !info) return fail(IVX_EINVAL, "plan and info must be non-NULL");
    const Geom &g = p->g;
    const int64_t v[16] = {g.nf, g.W, g.T, p->n_work, p->m_live, p->n_slots, (int64_t)p->dev_bytes,
                           (int64_t)g.C * g.P, g.eh, g.ew, p->graph_nodes, g.win, p->nwave, p->chunk_max, p->lanes, p->vpi};
    std::memcpy(info, v, sizeof(v));
    return IVX_OK;
}

ivx_status ivx_plan_set_data(ivx_plan *p, const ivx_real *uv, const ivx_real *vis, const ivx_real *weight,
                             const uint8_t *flags, const ivx_real *beams, const ivx_real *interp,
                             const ivx_real *sd_map, void *stream) {
    g_last_error.clear();
    if (!p) return fail(IVX_EINVAL, "plan is NULL");
    VisSource src;
    src.uv = uv;
    src.vis = vis;
    src.w = weight;
    src.flags = flags;
    return set_data_impl(p, src, false, beams, interp, sd_map, stream);
}

ivx_status ivx_plan_set_data_shared(ivx_plan *p, const ivx_real *uv, const ivx_real *weight, const double *uv_scale,
                                    const ivx_real *vis, const uint8_t *flags, const ivx_real *beams,
                                    const ivx_real *interp, const ivx_real *sd_map, void *stream) {
    g_last_error.clear();
    if (!p) return fail(IVX_EINVAL, "plan is NULL");
    if (!uv_scale) return fail(IVX_EINVAL, "uv_scale is required");
    for (int c = 0; c < p->g.C; ++c)
        if (!std::isfinite(uv_scale[c]) || !(uv_scale[c] > 0.0))
            return fail(IVX_EINVAL, "uv_scale must be finite and positive");
    for (int k = 0; k < p->g.P; ++k) {
        const int64_t m0 = p->offsets[(size_t)k * p->g.C + 1] - p->offsets[(size_t)k * p->g.C];
        for (int c = 1; c < p->g.C; ++c) {
            const int64_t b = (int64_t)k * p->g.C + c;
            if (p->offsets[b + 1] - p->offsets[b] != m0)
                return fail(IVX_EINVAL, "shared uv needs the same visibility count in every channel of a pointing");
        }
    }
    VisSource src;
    src.uv = uv;
    src.vis = vis;
    src.w = weight;
    src.flags = flags;
    src.scale = uv_scale;
    return set_data_impl(p, src, true, beams, interp, sd_map, stream);
}

ivx_status ivx_plan_set_w(ivx_plan *p, const ivx_real *w, int32_t w_width, double w_sigma, void *stream) {
    g_last_error.clear();
    if (!p) return fail(IVX_EINVAL, "plan is NULL");
    if (!p->has_data) return fail(IVX_ESTATE, "ivx_plan_set_data has not succeeded on this plan");
    drop_graph(p);
    ++p->epoch;
    if (!w) {
        p->w_on = false;
        return IVX_OK;
    }
    const int Ww = w_width ? w_width : std::max(p->g.W, 8);
    const double sigma = w_sigma != 0.0 ? w_sigma : 2.0;
    if (Ww < 2 || Ww > 16) return fail(IVX_EINVAL, "w_width must be 0 or in [2, 16]");
    if (!std::isfinite(sigma) || sigma < 1.25 || sigma > 8.0) return fail(IVX_EINVAL, "w_sigma must be 0 or in [1.25, 8]");
    hipStream_t st = (hipStream_t)stream;
    IVX_HIP(hipStreamSynchronize(st));
    p->w_on = false;
    ivx_status s = w_tables(p, Ww, sigma);
    if (s != IVX_OK) return s;
    const int64_t n = p->shared_uv ? p->pt_off.back() : p->m_total;
    if (!p->d_wsrc && (s = dalloc(p, &p->d_wsrc, (size_t)std::max<int64_t>(n, 1))) != IVX_OK) return s;
    if (n > 0) IVX_HIP(hipMemcpy(p->d_wsrc, w, n * sizeof(real), hipMemcpyDefault));
    p->w_on = true;
    p->w_version = ~0ull;
    if ((s = w_prepare(p, st)) != IVX_OK) {
        p->w_on = false;
        return s;
    }
    return IVX_OK;
}

ivx_status ivx_plan_w_info(const ivx_plan *p, double *info) {
    if (!p || !info) return fail(IVX_EINVAL, "plan and info must be non-NULL");
    const double v[6] = {p->w_on ? 1.0 : 0.0, (double)p->w_planes, p->w_dw, p->w_xc, (double)p->w_W, p->w_sigma};
    std::memcpy(info, v, sizeof(v));
    return IVX_OK;
}

} // extern "C"

namespace {

ivx_status set_data_impl(ivx_plan *p, const VisSource &src, bool shared, const ivx_real *beams,
                         const ivx_real *interp, const ivx_real *sd_map, void *stream) {
    const int64_t M = p->m_total;
    if (M > 0 && (!src.uv || !src.vis || !src.w)) return fail(IVX_EINVAL, "uv, vis and weight are required");
    if (!beams || !interp) return fail(IVX_EINVAL, "beams and interp are required");
    if (sd_active(p) && !sd_map) return fail(IVX_EINVAL, "sd_map is required when lambda_s > 0 and sd_n > 0");
    hipStream_t st = (hipStream_t)stream;
    IVX_HIP(hipStreamSynchronize(st));
    const Geom &g = p->g;
    const int n_items = g.C * g.P;
    const int64_t nk2 = (int64_t)g.nk * g.nk;
    // ---- host copies of the small per-pointing and single-dish arrays
    std::vector<real> h_beams(g.P * nk2), h_interp(g.P * nk2 * 2);
    IVX_HIP(hipMemcpy(h_beams.data(), beams, h_beams.size() * sizeof(real), hipMemcpyDefault));
    IVX_HIP(hipMemcpy(h_interp.data(), interp, h_interp.size() * sizeof(real), hipMemcpyDefault));
    std::vector<real> h_sd;
    if (sd_active(p)) {
        h_sd.resize((size_t)g.C * p->d.sd_n * p->d.sd_n);
        IVX_HIP(hipMemcpy(h_sd.data(), sd_map, h_sd.size() * sizeof(real), hipMemcpyDefault));
        for (real v : h_sd)
            if (!std::isfinite((double)v)) return fail(IVX_ENONFINITE, "sd_map holds a non-finite value");
    }
    for (size_t i = 0; i < h_beams.size(); ++i)
        if (!std::isfinite((double)h_beams[i])) return fail(IVX_ENONFINITE, "beams hold a non-finite value");
    free_all(p);
    ++p->epoch;
    p->shared_uv = shared;
    p->uv_scale.clear();
    if (shared) p->uv_scale.assign(src.scale, src.scale + g.C);
    p->pt_off.assign(g.P + 1, 0);
    for (int k = 0; k < g.P; ++k)
        p->pt_off[k + 1] = p->pt_off[k] + (p->offsets[(size_t)k * g.C + 1] - p->offsets[(size_t)k * g.C]);
    ivx_status s;
    // ---- constant tables and images
    if ((s = dalloc(p, &p->d_dq, g.nk)) != IVX_OK) goto fail_free;
    if ((s = dalloc(p, &p->d_fscale, g.C)) != IVX_OK) goto fail_free;
    if ((s = dalloc(p, &p->d_tw, g.nf)) != IVX_OK) goto fail_free;
    if ((s = dalloc(p, &p->d_beams, h_beams.size())) != IVX_OK) goto fail_free;
    if ((s = dalloc(p, &p->d_interp, h_interp.size())) != IVX_OK) goto fail_free;
    if ((s = dalloc(p, &p->d_R, (size_t)n_items * g.r_stride)) != IVX_OK) goto fail_free;
    if ((s = dalloc(p, &p->d_gp, (size_t)n_items * nk2)) != IVX_OK) goto fail_free;
    if ((s = dalloc(p, &p->d_terms, 5)) != IVX_OK) goto fail_free;
    p->n_rpart = sky_blocks(g);
    if ((s = dalloc(p, &p->d_rpart, p->n_rpart)) != IVX_OK) goto fail_free;
    if ((s = dalloc(p, &p->d_npart, p->n_rpart)) != IVX_OK) goto fail_free;
    {
        std::vector<real> fs(g.C);
        for (int c = 0; c < g.C; ++c) fs[c] = (real)p->fscale[c];
        hipError_t e;
        if ((e = hipMemcpy(p->d_dq, p->dq_host.data(), g.nk * sizeof(real), hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(p->d_fscale, fs.data(), g.C * sizeof(real), hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(p->d_tw, p->tw_host.data(), g.nf * sizeof(cpx), hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(p->d_beams, h_beams.data(), h_beams.size() * sizeof(real), hipMemcpyHostToDevice)) !=
                hipSuccess ||
            (e = hipMemcpy(p->d_interp, h_interp.data(), h_interp.size() * sizeof(real), hipMemcpyHostToDevice)) !=
                hipSuccess) {
            s = hip_fail(e, "hipMemcpy (set_data tables)");
            goto fail_free;
        }
    }
    // ---- transpose of the bilinear reprojection, pixel-major (fixed summation order)
    {
        const int N = g.N;
        std::vector<int32_t> cptr((size_t)N * N + 1, 0);
        struct Tap { int64_t pix; CsrEnt e; };
        std::vector<Tap> taps;
        taps.reserve((size_t)g.P * nk2 * 4);
        const int64_t koff = (int64_t)g.C * nk2;
        if (koff * g.P > INT32_MAX) { s = fail(IVX_EINVAL, "sub-image index exceeds int32"); goto fail_free; }
        for (int k = 0; k < g.P; ++k) {
            for (int64_t ab = 0; ab < nk2; ++ab) {
                const real sy = h_interp[((int64_t)k * nk2 + ab) * 2], sx = h_interp[((int64_t)k * nk2 + ab) * 2 + 1];
                if (!std::isfinite((double)sy) || !std::isfinite((double)sx)) continue;
                if (!(sy > real(-1) && sy < real(N) && sx > real(-1) && sx < real(N))) continue;
                const real fi = std::floor(sy), fj = std::floor(sx);
                const int i0 = (int)fi, j0 = (int)fj;
                const real fy = sy - fi, fx = sx - fj;
                const real wts[4] = {(real(1) - fy) * (real(1) - fx), (real(1) - fy) * fx, fy * (real(1) - fx), fy * fx};
                const int di[4] = {0, 0, 1, 1}, dj[4] = {0, 1, 0, 1};
                for (int t = 0; t < 4; ++t) {
                    const int ii = i0 + di[t], jj = j0 + dj[t];
                    if (ii < 0 || ii >= N || jj < 0 || jj >= N || wts[t] == real(0)) continue;
                    taps.push_back(Tap{(int64_t)ii * N + jj, CsrEnt{(int32_t)(k * koff + ab), wts[t]}});
                }
            }
        }
        for (const Tap &t : taps) cptr[t.pix + 1]++;
        for (int64_t i = 0; i < (int64_t)N * N; ++i) cptr[i + 1] += cptr[i];
        if ((int64_t)taps.size() > INT32_MAX) { s = fail(IVX_EINVAL, "too many reprojection taps"); goto fail_free; }
        std::vector<CsrEnt> cent(taps.size() > 0 ? taps.size() : 1);
        {
            std::vector<int32_t> fillp(cptr.begin(), cptr.end() - 1);
            for (const Tap &t : taps) cent[fillp[t.pix]++] = t.e; // stable: (k, a, b, tap) order
        }
        // sliced layout for the sky pass: one slice per wave of its 16 x 16 pixel blocks
        // (4 rows of 16 pixels), entries stored entry-major within the slice (lane-
        // contiguous) and padded to the slice's longest pixel with zero weights
        const int nb = (N + SKY_T - 1) / SKY_T;
        const int64_t nslice = (int64_t)nb * nb * (SKY_T * SKY_T / 64);
        std::vector<int32_t> soff(nslice + 1, 0);
        auto slice_pixel = [&](int64_t sl, int lane, int64_t &pix) {
            const int64_t blk = sl / (SKY_T * SKY_T / 64);
            const int w = (int)(sl % (SKY_T * SKY_T / 64));
            const int by = (int)(blk / nb), bx = (int)(blk % nb);
            const int tid = w * 64 + lane;
            const int i = by * SKY_T + tid / SKY_T, j = bx * SKY_T + tid % SKY_T;
            if (i >= N || j >= N) return false;
            pix = (int64_t)i * N + j;
            return true;
        };
        int64_t tot = 0;
        for (int64_t sl = 0; sl < nslice; ++sl) {
            int len = 0;
            for (int lane = 0; lane < 64; ++lane) {
                int64_t pix;
                if (slice_pixel(sl, lane, pix)) len = std::max(len, cptr[pix + 1] - cptr[pix]);
            }
            soff[sl] = (int32_t)tot;
            tot += (int64_t)len * 64;
            if (tot > INT32_MAX) { s = fail(IVX_EINVAL, "too many reprojection taps"); goto fail_free; }
        }
        soff[nslice] = (int32_t)tot;
        std::vector<CsrEnt> sell(tot > 0 ? tot : 1, CsrEnt{0, real(0)});
        for (int64_t sl = 0; sl < nslice; ++sl)
            for (int lane = 0; lane < 64; ++lane) {
                int64_t pix;
                if (!slice_pixel(sl, lane, pix)) continue;
                for (int t = 0; t < cptr[pix + 1] - cptr[pix]; ++t) sell[soff[sl] + (int64_t)t * 64 + lane] = cent[cptr[pix] + t];
            }
        if ((s = dalloc(p, &p->d_cptr, soff.size())) != IVX_OK) goto fail_free;
        if ((s = dalloc(p, &p->d_cent, sell.size())) != IVX_OK) goto fail_free;
        hipError_t e;
        if ((e = hipMemcpy(p->d_cptr, soff.data(), soff.size() * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(p->d_cent, sell.data(), sell.size() * sizeof(CsrEnt), hipMemcpyHostToDevice)) != hipSuccess) {
            s = hip_fail(e, "hipMemcpy (reprojection transpose)");
            goto fail_free;
        }
    }
    // ---- single dish
    if (sd_active(p)) {
        const int sdn = p->d.sd_n;
        p->n_kpart = (int)(((int64_t)g.C * sdn * sdn + 255) / 256);
        if ((s = dalloc(p, &p->d_sdmap, h_sd.size())) != IVX_OK) goto fail_free;
        if ((s = dalloc(p, &p->d_gB, p->gB_host.size())) != IVX_OK) goto fail_free;
        if ((s = dalloc(p, &p->d_U, (size_t)g.C * g.N * sdn)) != IVX_OK) goto fail_free;
        if ((s = dalloc(p, &p->d_E, (size_t)g.C * sdn * sdn)) != IVX_OK) goto fail_free;
        if ((s = dalloc(p, &p->d_kpart, p->n_kpart)) != IVX_OK) goto fail_free;
        hipError_t e;
        if ((e = hipMemcpy(p->d_sdmap, h_sd.data(), h_sd.size() * sizeof(real), hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(p->d_gB, p->gB_host.data(), p->gB_host.size() * sizeof(real), hipMemcpyHostToDevice)) !=
                hipSuccess) {
            s = hip_fail(e, "hipMemcpy (single dish)");
            goto fail_free;
        }
    }
    if ((s = dalloc(p, &p->d_boff, (size_t)n_items + 1)) != IVX_OK) goto fail_free;
    {
        hipError_t e = hipMemcpy(p->d_boff, p->offsets.data(), ((size_t)n_items + 1) * sizeof(int64_t),
                                 hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            s = hip_fail(e, "hipMemcpy (block offsets)");
            goto fail_free;
        }
    }
    if ((s = bin_from_caller(p, src, st)) != IVX_OK || (s = build_work(p, st)) != IVX_OK) goto fail_free;
    p->has_data = true;
    return IVX_OK;
fail_free:
    {
        const std::string msg = g_last_error;
        free_all(p);
        g_last_error = msg;
    }
    return s;
}

} // namespace

extern "C" {

ivx_status ivx_plan_set_vis(ivx_plan *p, const ivx_real *vis, const ivx_real *weight, void *stream) {
    ivx_status s = check_plan_use(p);
    if (s != IVX_OK) return s;
    if (!vis && p->m_total > 0) return fail(IVX_EINVAL, "vis is required");
    hipStream_t st = (hipStream_t)stream;
    const Geom &g = p->g;
    const int n_items = g.C * g.P;
    const bool vis_dev = on_device(vis), w_dev = on_device(weight);
    int64_t maxn = 0, maxw = 0;
    for (int b = 0; b < n_items; ++b) maxn = std::max(maxn, p->offsets[b + 1] - p->offsets[b]);
    if (p->shared_uv)
        for (int k = 0; k < g.P; ++k) maxw = std::max(maxw, p->pt_off[k + 1] - p->pt_off[k]);
    else
        maxw = maxn;
    TmpBuf bad, s_vis, s_w;
    IVX_HIP(bad.get(sizeof(unsigned int)));
    if (!vis_dev) IVX_HIP(s_vis.get(2 * maxn * sizeof(real)));
    if (weight && !w_dev) IVX_HIP(s_w.get(maxw * sizeof(real)));
    IVX_HIP(hipMemsetAsync(bad.p, 0, sizeof(unsigned int), st));
    int staged_k = -1;
    const real *wb = nullptr;
    for (int b = 0; b < n_items; ++b) {
        const int64_t L0 = p->block_live[b], n = p->block_live[b + 1] - L0;
        if (n == 0) continue;
        const int k = b / g.C;
        const int64_t off = p->offsets[b], nb = p->offsets[b + 1] - off;
        const real *vb = nullptr;
        if ((s = block_view(vis, vis_dev, 2 * off, 2 * nb, s_vis, &vb, st)) != IVX_OK) return s;
        if (weight) {
            if (p->shared_uv) {
                if (k != staged_k) {
                    const int64_t po = p->pt_off[k], pn = p->pt_off[k + 1] - po;
                    if ((s = block_view(weight, w_dev, po, pn, s_w, &wb, st)) != IVX_OK) return s;
                    staged_k = k;
                }
            } else if ((s = block_view(weight, w_dev, off, nb, s_w, &wb, st)) != IVX_OK) {
                return s;
            }
        }
        IVX_HIP(launch_gather_block(n, p->d_perm + L0, vb, weight ? wb : nullptr, p->d_vis + L0, p->d_wgt + L0,
                                    bad.as<unsigned int>(), st));
    }
    unsigned int hb = 0;
    IVX_HIP(hipMemcpyAsync(&hb, bad.p, sizeof(unsigned int), hipMemcpyDeviceToHost, st));
    IVX_HIP(hipStreamSynchronize(st));
    if (hb) return fail(IVX_ENONFINITE, "ivx_plan_set_vis: non-finite value or negative weight");
    return IVX_OK;
}

ivx_status ivx_objective_grad(ivx_plan *p, const ivx_real *sky, ivx_real *grad, double *terms, void *stream) {
    ivx_status s = check_plan_use(p);
    if (s != IVX_OK) return s;
    if (!sky || !grad) return fail(IVX_EINVAL, "sky and grad are required");
    hipStream_t st = (hipStream_t)stream;
    // device `terms` is written by the last kernel itself; host `terms` gets a copy
    double *terms_dev = device_terms(terms);
    if (p->w_on) { // full model: eager launches, one pass per w plane
        if ((s = w_prepare(p, st)) != IVX_OK) return s;
        if ((s = eval_value_w(p, sky, terms_dev, true, st)) != IVX_OK) return s;
        if ((s = eval_gradient_w(p, sky, grad, real(1), st)) != IVX_OK) return s;
        return copy_terms(p, terms, terms_dev, st);
    }
    if (p->use_graph && p->timing_mask == 0) {
        if (!(p->gexec && p->g_sky == sky && p->g_grad == grad && p->g_terms == terms_dev)) {
            drop_graph(p);
            if (!p->cap_stream) IVX_HIP(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
            IVX_HIP(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
            ivx_status cs = eval_objective(p, sky, grad, terms_dev, p->cap_stream);
            hipGraph_t graph = nullptr;
            hipError_t ee = hipStreamEndCapture(p->cap_stream, &graph);
            if (cs != IVX_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return cs;
            }
            if (ee != hipSuccess) return hip_fail(ee, "hipStreamEndCapture");
            size_t nn = 0;
            (void)hipGraphGetNodes(graph, nullptr, &nn);
            hipError_t ie = hipGraphInstantiate(&p->gexec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ie != hipSuccess) {
                p->gexec = nullptr;
                return hip_fail(ie, "hipGraphInstantiate");
            }
            p->g_sky = sky;
            p->g_grad = grad;
            p->g_terms = terms_dev;
            p->graph_nodes = (int64_t)nn;
        }
        IVX_HIP(hipGraphLaunch(p->gexec, st));
    } else {
        if ((s = eval_objective(p, sky, grad, terms_dev, st)) != IVX_OK) return s;
    }
    return copy_terms(p, terms, terms_dev, st);
}

ivx_status ivx_forward(ivx_plan *p, const ivx_real *sky, ivx_real *model_vis, void *stream) {
    ivx_status s = check_plan_use(p);
    if (s != IVX_OK) return s;
    if (!sky || (!model_vis && p->m_total > 0)) return fail(IVX_EINVAL, "sky and model_vis are required");
    hipStream_t st = (hipStream_t)stream;
    if (p->w_on) {
        if ((s = w_prepare(p, st)) != IVX_OK || (s = w_forward_planes(p, sky, st)) != IVX_OK) return s;
        IVX_HIP(launch_zero(model_vis, p->m_total * 2 * (int64_t)sizeof(real), st));
        IVX_HIP(launch_wout(p->d_work, p->n_work, wgeom(p), p->d_wz, p->d_perm, p->d_boff, p->d_wacc,
                            reinterpret_cast<cpx *>(model_vis), st));
        return IVX_OK;
    }
    if ((s = run_forward_half(p, sky, st)) != IVX_OK) return s;
    IVX_HIP(launch_zero(model_vis, p->m_total * 2 * (int64_t)sizeof(real), st));
    IVX_HIP(launch_grid(MODE_FWD, p->g, p->d_work, p->n_work, p->d_crd, p->d_vis, p->d_wgt, p->d_perm, p->d_boff, p->d_ext,
                        p->d_slots, p->d_jpart, nullptr, reinterpret_cast<cpx *>(model_vis), p->nwave, p->lanes * 10 + p->vpi, p->occupancy, st));
    return IVX_OK;
}

ivx_status ivx_adjoint(ivx_plan *p, const ivx_real *vis, ivx_real *image, void *stream) {
    ivx_status s = check_plan_use(p);
    if (s != IVX_OK) return s;
    if (!image || (!vis && p->m_total > 0)) return fail(IVX_EINVAL, "vis and image are required");
    hipStream_t st = (hipStream_t)stream;
    if (p->w_on) return w_adjoint_call(p, vis, image, false, st);
    IVX_HIP(launch_grid(MODE_ADJ, p->g, p->d_work, p->n_work, p->d_crd, p->d_vis, p->d_wgt, p->d_perm, p->d_boff, p->d_ext,
                        p->d_slots, p->d_jpart, reinterpret_cast<const cpx *>(vis), nullptr, p->nwave, p->lanes * 10 + p->vpi, p->occupancy, st));
    if ((s = run_adjoint_half(p, st)) != IVX_OK) return s;
    IVX_HIP(launch_sky(p->g, image, p->d_gp, p->d_cptr, p->d_cent, real(0), real(0), nullptr, nullptr, 0, 0, 1, 0,
                       image, p->d_rpart, SKY_ADJOINT, real(1), st));
    return IVX_OK;
}

ivx_status ivx_objective(ivx_plan *p, const ivx_real *sky, double *terms, void *stream) {
    ivx_status s = check_plan_use(p);
    if (s != IVX_OK) return s;
    if (!sky || !terms) return fail(IVX_EINVAL, "sky and terms are required");
    hipStream_t st = (hipStream_t)stream;
    double *terms_dev = device_terms(terms);
    if (p->w_on) {
        if ((s = w_prepare(p, st)) != IVX_OK || (s = eval_value_w(p, sky, terms_dev, false, st)) != IVX_OK) return s;
    } else if ((s = eval_value(p, sky, terms_dev, MODE_VAL, st)) != IVX_OK) {
        return s;
    }
    return copy_terms(p, terms, terms_dev, st);
}

ivx_status ivx_objective_forward(ivx_plan *p, const ivx_real *sky, double *terms, void *stream) {
    ivx_status s = check_plan_use(p);
    if (s != IVX_OK) return s;
    if (!sky || !terms) return fail(IVX_EINVAL, "sky and terms are required");
    hipStream_t st = (hipStream_t)stream;
    double *terms_dev = device_terms(terms);
    if (p->w_on) {
        if ((s = w_prepare(p, st)) != IVX_OK || (s = eval_value_w(p, sky, terms_dev, true, st)) != IVX_OK) return s;
    } else if ((s = eval_value(p, sky, terms_dev, MODE_OBJ, st)) != IVX_OK) {
        return s;
    }
    p->fwd_epoch = p->epoch;
    p->fwd_sky = sky;
    return copy_terms(p, terms, terms_dev, st);
}

ivx_status ivx_objective_backward(ivx_plan *p, const ivx_real *sky, ivx_real *grad, double scale, void *stream) {
    ivx_status s = check_plan(p);
    if (s != IVX_OK) return s;
    if (!sky || !grad) return fail(IVX_EINVAL, "sky and grad are required");
    if (!std::isfinite(scale)) return fail(IVX_EINVAL, "scale must be finite");
    if (p->fwd_epoch != p->epoch || p->fwd_sky != sky)
        return fail(IVX_ESTATE, "ivx_objective_backward must follow ivx_objective_forward of the same sky with no "
                                "other call on the plan in between");
    ++p->epoch; // the adjoint half consumes the slots: a second backward needs a new forward
    if (p->w_on) return eval_gradient_w(p, sky, grad, (real)scale, (hipStream_t)stream);
    return eval_gradient(p, sky, grad, (real)scale, (hipStream_t)stream);
}

ivx_status ivx_forward_adjoint(ivx_plan *p, const ivx_real *vis, ivx_real *image, void *stream) {
    ivx_status s = check_plan_use(p);
    if (s != IVX_OK) return s;
    if (!image || (!vis && p->m_total > 0)) return fail(IVX_EINVAL, "vis and image are required");
    hipStream_t st = (hipStream_t)stream;
    if (p->w_on) return w_adjoint_call(p, vis, image, true, st);
    IVX_HIP(launch_grid(MODE_ADJ, p->g, p->d_work, p->n_work, p->d_crd, p->d_vis, p->d_wgt, p->d_perm, p->d_boff,
                        p->d_ext, p->d_slots, p->d_jpart, reinterpret_cast<const cpx *>(vis), nullptr, p->nwave,
                        p->lanes * 10 + p->vpi, p->occupancy, st, true));
    if ((s = run_adjoint_half(p, st)) != IVX_OK) return s;
    IVX_HIP(launch_sky(p->g, image, p->d_gp, p->d_cptr, p->d_cent, real(0), real(0), nullptr, nullptr, 0, 0, 1, 0,
                       image, p->d_rpart, SKY_ADJOINT, real(1), st));
    return IVX_OK;
}

ivx_status ivx_autotune(ivx_plan *p, double budget_ms, int32_t *chosen_tile, void *stream) {
    ivx_status s = check_plan_use(p);
    if (s != IVX_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    struct Cand { int W, nf, T, nwave, chunk, lanes, vpi; };
    // NUFFT geometries: the plan's own, and when the library chose it, the narrowest kernel on
    // the plan's fine grid and on the grids of half and twice its size whose accuracy probe
    // meets the plan's target (the requested nufft_eps, else the accuracy of the plan's own
    // geometry): the result stays as accurate as requested while the cost may change
    std::vector<std::pair<int, int>> geoms;
    if (p->geometry_auto) {
        for (int nf : {p->g.nf, p->g.nf / 2, p->g.nf * 2}) {
            if (nf < 64 || nf > 2048 || nf * 4 < p->g.nk * 5) continue;
            for (int W = 4; W <= 16; ++W) {
                if (nufft_probe_error(p->g.nk, nf, W) > p->eps_target) continue;
                geoms.push_back({W, nf});
                break;
            }
        }
    }
    // the plan's own geometry when it meets the target (a plan created with a width its
    // requested accuracy does not support is moved to one that does), or when it is fixed
    if (geoms.empty() || nufft_probe_error(p->g.nk, p->g.nf, p->g.W) <= p->eps_target) {
        bool have = false;
        for (const auto &gm : geoms) have = have || (gm.first == p->g.W && gm.second == p->g.nf);
        if (!have) geoms.insert(geoms.begin(), {p->g.W, p->g.nf});
    }
    const int tiles[] = {8, 12, 16, 24, 32};
    const int waves[] = {4, 2, 1};
    const int chunks[] = {128, 256, 512};
    auto blockings = [&](int W, int nf) {
        std::vector<Cand> c;
        // the matrix-core gridder first (one wave per work item, windows of at most 16 x 16):
        // it is the fastest where it fits, and the search may stop at the time budget
        for (int T = 17 - W; T >= W; --T)
            if (tile_fits(p, T, 1, GRID_MFMA_LANES))
                for (int ch : chunks) c.push_back(Cand{W, nf, T, 1, ch, GRID_MFMA_LANES, 1});
        for (int lanes : {16, 8})
            for (int vpi : {2, 1})
                for (int T : tiles)
                    for (int nw : waves)
                        if (tile_fits(p, T, nw, lanes))
                            for (int ch : chunks) c.push_back(Cand{W, nf, T, nw, ch, lanes, vpi});
        return c;
    };
    // whole evaluations at a zero sky on the plan's own data (the geometry changes the FFT
    // passes too); the fastest candidate is kept
    real *sky = nullptr, *grad = nullptr;
    const int64_t nsky = (int64_t)p->g.C * p->g.N * p->g.N;
    IVX_HIP(hipMalloc(&sky, nsky * sizeof(real)));
    if (hipMalloc(&grad, nsky * sizeof(real)) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(sky);
        return fail(IVX_ENOMEM, "autotune buffers");
    }
    IVX_HIP(hipMemsetAsync(sky, 0, nsky * sizeof(real), st));
    hipEvent_t e0, e1;
    IVX_HIP(hipEventCreate(&e0));
    IVX_HIP(hipEventCreate(&e1));
    const auto t_start = std::chrono::steady_clock::now();
    double best_ms = 1e300;
    Cand best{p->g.W, p->g.nf, p->g.T, p->nwave, p->chunk_max, p->lanes, p->vpi};
    const uint32_t mask = p->timing_mask;
    p->timing_mask = 0;
    bool out_of_time = false;
    for (const auto &gm : geoms) {
        if (out_of_time) break;
        if ((s = apply_geometry(p, gm.first, gm.second)) == IVX_ENOMEM) {
            s = IVX_OK; // this geometry does not fit next to the data: skip it
            continue;
        }
        if (s != IVX_OK) break;
        const int lanes0 = p->lanes;
        std::vector<Cand> cands = blockings(gm.first, gm.second);
        p->lanes = lanes0;
        for (const Cand &c : cands) {
            p->nwave = c.nwave;
            p->lanes = c.lanes;
            p->vpi = c.vpi;
            p->chunk_max = c.chunk;
            set_tile(p, c.T);
            if ((s = build_bins(p, st)) == IVX_ENOMEM) {
                s = IVX_OK; // this blocking does not fit next to the data: skip it
                continue;
            }
            if (s != IVX_OK) break;
            float ms = 0.f, tot = 0.f;
            const int reps = 3;
            for (int r = 0; r < reps + 1; ++r) {
                IVX_HIP(hipEventRecord(e0, st));
                if ((s = eval_objective(p, sky, grad, nullptr, st)) != IVX_OK) break;
                IVX_HIP(hipEventRecord(e1, st));
                IVX_HIP(hipEventSynchronize(e1));
                IVX_HIP(hipEventElapsedTime(&ms, e0, e1));
                if (r > 0) tot += ms;
            }
            if (s != IVX_OK) break;
            const double avg = tot / reps;
            if (avg < best_ms) {
                best_ms = avg;
                best = c;
            }
            const double spent =
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
            if (spent > budget_ms) {
                out_of_time = true;
                break;
            }
        }
        if (s != IVX_OK) break;
    }
    p->timing_mask = mask;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(sky);
    (void)hipFree(grad);
    if (s != IVX_OK) return s;
    if ((s = apply_geometry(p, best.W, best.nf)) != IVX_OK) return s;
    p->nwave = best.nwave;
    p->lanes = best.lanes;
    p->vpi = best.vpi;
    p->chunk_max = best.chunk;
    set_tile(p, best.T);
    if ((s = build_bins(p, st)) != IVX_OK) return s;
    if (chosen_tile) *chosen_tile = best.T;
    return IVX_OK;
}

extern "C" ivx_status ivx_nufft_probe(int32_t n_sub, int32_t n_fine, int32_t kernel_width, double *err) {
    if (!err || n_sub < 4 || (n_sub & 1) || n_fine < n_sub || kernel_width < 2 || kernel_width > 16)
        return fail(IVX_EINVAL, "bad ivx_nufft_probe arguments");
    *err = nufft_probe_error(n_sub, n_fine, kernel_width);
    return IVX_OK;
}

extern "C" ivx_status ivx_sort_u64(const uint64_t *keys_in, uint64_t *keys_out, const uint32_t *vals_in,
                                   uint32_t *vals_out, int64_t n, int32_t end_bit, void *stream) {
    if (n < 0 || n > (int64_t)INT32_MAX || end_bit < 1 || end_bit > 64)
        return fail(IVX_EINVAL, "ivx_sort_u64: n must be in [0, 2^31) and end_bit in [1, 64]");
    if (n == 0) return IVX_OK;
    if (!keys_in || !keys_out || (vals_in && !vals_out))
        return fail(IVX_EINVAL, "ivx_sort_u64: keys_in, keys_out (and vals_out with vals_in) are required");
    hipStream_t st = (hipStream_t)stream;
    const size_t bytes = radix_sort_temp_bytes((int)n, vals_in != nullptr);
    void *temp = nullptr;
    IVX_HIP(hipStreamSynchronize(st));
    IVX_HIP(hipMalloc(&temp, bytes));
    const hipError_t e = radix_sort(temp, bytes, keys_in, keys_out, vals_in, vals_in ? vals_out : nullptr, (int)n,
                                    end_bit, st);
    const hipError_t e2 = hipStreamSynchronize(st);
    (void)hipFree(temp);
    IVX_HIP(e);
    IVX_HIP(e2);
    return IVX_OK;
}

} // extern "C"
