/*
 * ivx_lbfgsb — the positivity-bounded quasi-Newton loop of Classic3D on the device.
 *
 * The paper minimises Q_tot over the sky cube with L-BFGS-B under x >= 0, starting from
 * x = 0 (Sect. 3.4, Eq. L-BFGS-B; the null prior of Sect. 2.2).  This solver runs that
 * method with every length-n vector operation on the GPU and only O(m^2) scalars on the
 * host, calling ivx_objective_grad of the plan for each function evaluation:
 *
 *   - compact limited-memory BFGS matrix B = theta I - W M W^T, W = [Y, theta S]
 *     (Byrd, Nocedal & Schnabel 1994), FP64 state (x, g, S, Y) in device memory;
 *   - generalized Cauchy point along the projected steepest-descent path (Byrd, Lu,
 *     Nocedal & Zhu 1995): breakpoints sorted on the device and the sequential f'/f''
 *     recurrence of the method evaluated for all breakpoints at once with prefix sums;
 *   - subspace minimisation over the free variables (direct primal method) with the
 *     projected step and its truncated fall-back (Morales & Nocedal 2011);
 *   - strong-Wolfe line search of More & Thuente (1994) along d = xbar - x
 *     (ftol 1e-3, gtol 0.9, xtol 0.1, at most maxls evaluations);
 *   - memory update skipped unless s^T y > eps (-g^T s); a failed line search discards
 *     the memory and retries from the last iterate.
 *
 * Stopping rules follow scipy's L-BFGS-B defaults: projected-gradient infinity norm
 * <= gtol, relative reduction (f_k - f_{k+1}) / max(|f_k|, |f_{k+1}|, 1) <= ftol, or the
 * iteration / evaluation caps; in addition, an optional target stops at the first
 * evaluation with f <= target (time-to-tolerance).
 *
 * The objective is evaluated in the plan's precision (ivx_real) at the FP64 iterate
 * rounded to ivx_real; all solver arithmetic is FP64.  Status codes and ivx_last_error()
 * are those of ivx.h.
 */
#ifndef IVX_LBFGSB_H
#define IVX_LBFGSB_H

#include <stdint.h>

#include "ivx.h"

#ifdef __cplusplus
extern "C" {
#endif

#define IVX_LBFGSB_MAX_M 16

typedef struct ivx_lbfgsb ivx_lbfgsb;

typedef struct {
    int32_t m;           /* correction pairs kept, 1..IVX_LBFGSB_MAX_M (10) */
    int32_t maxiter;     /* iteration cap (15000) */
    int32_t maxfun;      /* objective-evaluation cap (15000) */
    int32_t maxls;       /* evaluations per line search (20) */
    int32_t positivity;  /* 1: x >= 0 componentwise (the paper's bound); 0: unbounded (1) */
    int32_t full_sort;   /* 1: every Cauchy search sorts all breakpoints; 0: first only those
                            below a sampled threshold, in one workgroup, and all of them only
                            when the minimiser lies beyond (same iterates either way; problems of
                            more than 2^24 variables always sort all) (0) */
    int32_t stream_wait; /* 1: the host reads each step's results after the stream has drained;
                            0: as soon as the step's last kernel has published them, by spinning
                            on a sequence number it writes into the mapped host buffer, falling
                            back to the stream wait after 20 ms (same iterates either way) (0) */
    int32_t reserved;    /* 0 */
    double ftol;         /* relative-reduction tolerance (2.220446049250313e-09) */
    double gtol;         /* projected-gradient infinity-norm tolerance (1e-5) */
    double target;       /* stop once f <= target; -INFINITY disables (-INFINITY) */
} ivx_lbfgsb_options;

typedef enum {
    IVX_LBFGSB_PGTOL = 0,     /* projected gradient below gtol */
    IVX_LBFGSB_FTOL = 1,      /* relative reduction below ftol */
    IVX_LBFGSB_MAXITER = 2,
    IVX_LBFGSB_MAXFUN = 3,
    IVX_LBFGSB_TARGET = 4,    /* an evaluation reached opt.target */
    IVX_LBFGSB_ABNORMAL = 5   /* line search failed with an empty memory */
} ivx_lbfgsb_reason;

typedef struct {
    double f;            /* objective at the returned x */
    double pg_norm;      /* projected-gradient infinity norm at the returned x */
    int64_t nit;         /* iterations */
    int64_t nfev;        /* objective evaluations */
    int32_t reason;      /* ivx_lbfgsb_reason */
    int32_t n_walks_full; /* of n_walks, those that sorted all breakpoints */
    int64_t n_walks;     /* Cauchy searches that crossed at least one breakpoint (sorted path) */
} ivx_lbfgsb_result;

/* Fill `opt` with the defaults above. */
ivx_status ivx_lbfgsb_default_options(ivx_lbfgsb_options *opt);

/* Solver workspace for `plan` (n = n_chan * n_sky^2 variables) with up to m_max
 * correction pairs: allocates about (2 m_max + 100) * n * 8 bytes of device memory and a
 * small pinned host buffer.  The plan must outlive the solver. */
ivx_status ivx_lbfgsb_create(ivx_plan *plan, int32_t m_max, ivx_lbfgsb **out);
ivx_status ivx_lbfgsb_destroy(ivx_lbfgsb *solver);

/* Minimise the plan's Q_tot from x (device, [n_chan][n_sky][n_sky] ivx_real: the start on
 * entry, projected onto the bounds; the last accepted iterate on return, or the
 * evaluation that reached the target).  opt NULL = defaults (opt->m <= m_max).
 * f_history / t_history (host, may be NULL) receive Q_tot and the seconds since the call
 * began for the first history_capacity evaluations.  Synchronous on `stream` (the loop
 * reads a few scalars back per step); res (host) is required. */
ivx_status ivx_lbfgsb_solve(ivx_lbfgsb *solver, ivx_real *x, const ivx_lbfgsb_options *opt,
                            double *f_history, double *t_history, int64_t history_capacity,
                            ivx_lbfgsb_result *res, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* IVX_LBFGSB_H */
