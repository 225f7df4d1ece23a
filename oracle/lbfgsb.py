"""Plain FP64 CPU L-BFGS-B — TEST INFRASTRUCTURE (oracle of the bounded quasi-Newton loop).

The paper minimises Q_tot with L-BFGS-B under x >= 0 (Sect. 3.4, Eq. L-BFGS-B).  This is a
direct, unoptimised statement of that method for lower bounds (upper bounds infinite),
written from the published descriptions, with dense small matrices and sequential loops:

* compact limited-memory matrix  B = theta I - W M W^T,  W = [Y, theta S],
  M = [[-D, L^T], [L, theta S^T S]]^-1                    (Byrd, Nocedal, Schnabel 1994)
* generalized Cauchy point: the first local minimiser of the quadratic model along the
  projected steepest-descent path, breakpoints visited in increasing order, f' and f''
  updated with the compact form                         (Byrd, Lu, Nocedal, Zhu 1995, Alg. CP)
* subspace minimisation over the free variables by the direct primal method, and the
  projection of its step onto the box with a fall-back to the truncated step when the
  projected point is not a descent direction           (same, Sect. 5.1; Morales & Nocedal 2011)
* line search along d = xbar - x satisfying the strong Wolfe conditions with the
  safeguarded cubic/quadratic interpolation of More & Thuente (1994), ftol 1e-3, gtol 0.9,
  xtol 0.1; first iteration starts at min(1/||d||, max feasible step), later ones at 1
* memory update skipped unless s^T y > eps * (-g^T s); a failed line search discards the
  memory and retries from the last iterate
* stop on the projected-gradient infinity norm <= gtol, a relative reduction
  (f_k - f_{k+1}) / max(|f_k|, |f_{k+1}|, 1) <= ftol, or an iteration / evaluation cap.

Pinned in tests/test_lbfgsb_oracle.py against brute force (the Cauchy point by exhaustive
piecewise minimisation of the dense quadratic model, the subspace step by a dense solve)
and against scipy.optimize's L-BFGS-B (iterates and solutions).
"""
from __future__ import annotations

import math

import numpy as np

EPS = float(np.finfo(np.float64).eps)


def projected_gradient_norm(x, g, lower):
    """|| P(x - g) - x ||_inf for the bounds x >= lower."""
    return float(np.max(np.abs(np.maximum(x - g, lower) - x))) if x.size else 0.0


# --------------------------------------------------------------------- compact form
def middle_matrix(S, Y, theta):
    """M for the stored pairs S, Y (n x k, oldest first)."""
    k = S.shape[1]
    if k == 0:
        return np.zeros((0, 0))
    SY = S.T @ Y
    D = np.diag(np.diag(SY))
    L = np.tril(SY, -1)
    K = np.block([[-D, L.T], [L, theta * (S.T @ S)]])
    return np.linalg.inv(K)


def dense_B(S, Y, theta):
    n = S.shape[0]
    W = np.hstack([Y, theta * S])
    return theta * np.eye(n) - W @ middle_matrix(S, Y, theta) @ W.T


# --------------------------------------------------------------------- Cauchy point
def cauchy_point(x, g, lower, theta, W, M):
    """Generalized Cauchy point.  Returns (xc, c, free) with c = W^T (xc - x) and `free`
    the variables not fixed at a bound by the search."""
    n = x.size
    t = np.full(n, np.inf)
    pos = g > 0
    t[pos] = (x[pos] - lower[pos]) / g[pos]
    d = np.where(t == 0.0, 0.0, -g)
    fixed = t == 0.0
    xc = x.copy()
    p = W.T @ d
    c = np.zeros(W.shape[1])
    fp = -float(d @ d)
    fpp = -theta * fp - float(p @ M @ p)
    fpp0 = fpp
    dtm = -fp / fpp if fpp > 0 else 0.0
    order = [i for i in np.argsort(t, kind="stable") if 0.0 < t[i] < np.inf]
    told = 0.0
    k = 0
    if fp >= 0:
        return x.copy(), c, ~fixed
    while k < len(order):
        b = order[k]
        dt = t[b] - told
        if dtm < dt:
            break
        # variable b reaches its bound
        xc[b] = lower[b]
        zb = lower[b] - x[b]
        c = c + dt * p
        gb = g[b]
        wb = W[b]
        fp = fp + dt * fpp + gb * gb + theta * gb * zb - gb * float(wb @ M @ c)
        fpp = fpp - theta * gb * gb - 2.0 * gb * float(wb @ M @ p) - gb * gb * float(wb @ M @ wb)
        fpp = max(EPS * fpp0, fpp)
        p = p + gb * wb
        d[b] = 0.0
        fixed[b] = True
        told = t[b]
        dtm = -fp / fpp
        k += 1
    dtm = max(dtm, 0.0)
    tc = told + dtm
    free = ~fixed
    xc[free] = x[free] + tc * d[free]
    c = c + dtm * p
    return xc, c, free


# ----------------------------------------------------------------- subspace step
def subspace_step(x, xc, g, lower, theta, W, M, c, free):
    """Minimise the quadratic model over the free variables from xc (direct primal
    method), then project onto the box; fall back to the longest feasible fraction of the
    step when the projected point is not a descent direction.  Returns xbar."""
    if W.shape[1] == 0 or not free.any():
        return xc.copy()
    du = subspace_direction(x, xc, g, theta, W, M, c, free)
    xbar = xc.copy()
    xbar[free] = np.maximum(xc[free] + du, lower[free])
    if float((xbar - x) @ g) < 0.0:
        return xbar
    alpha = 1.0
    neg = du < 0
    if neg.any():
        alpha = min(1.0, float(np.min((lower[free][neg] - xc[free][neg]) / du[neg])))
    xbar = xc.copy()
    xbar[free] = xc[free] + alpha * du
    return xbar


# -------------------------------------------------------------------- line search
class MoreThuente:
    """Strong-Wolfe line search of More & Thuente (1994) as a state machine: call
    start(f0, g0, stp) once, then step(f, g) after every evaluation at self.stp until
    it returns "conv" or "warn"."""

    XTRAPL, XTRAPU = 1.1, 4.0

    def __init__(self, ftol=1e-3, gtol=0.9, xtol=0.1, stpmin=0.0, stpmax=1e10):
        self.ftol, self.gtol, self.xtol = ftol, gtol, xtol
        self.stpmin, self.stpmax = stpmin, stpmax

    def start(self, f0, g0, stp):
        self.bracketed = False
        self.stage = 1
        self.finit, self.ginit = f0, g0
        self.gtest = self.ftol * g0
        self.width = self.stpmax - self.stpmin
        self.width1 = 2.0 * self.width
        self.stx, self.fx, self.gx = 0.0, f0, g0
        self.sty, self.fy, self.gy = 0.0, f0, g0
        self.stmin = 0.0
        self.stmax = stp + self.XTRAPU * stp
        self.stp = stp

    def step(self, f, g):
        stp = self.stp
        ftest = self.finit + stp * self.gtest
        if self.stage == 1 and f <= ftest and g >= 0.0:
            self.stage = 2
        if self.bracketed and (stp <= self.stmin or stp >= self.stmax):
            return "warn"
        if self.bracketed and self.stmax - self.stmin <= self.xtol * self.stmax:
            return "warn"
        if stp == self.stpmax and f <= ftest and g <= self.gtest:
            return "warn"
        if stp == self.stpmin and (f > ftest or g >= self.gtest):
            return "warn"
        if f <= ftest and abs(g) <= self.gtol * (-self.ginit):
            return "conv"
        if self.stage == 1 and f <= self.fx and f > ftest:
            gt = self.gtest
            fx, gx = self.fx - self.stx * gt, self.gx - gt
            fy, gy = self.fy - self.sty * gt, self.gy - gt
            fm, gm = f - stp * gt, g - gt
            (self.stx, fx, gx, self.sty, fy, gy, nstp) = self._interpolate(
                self.stx, fx, gx, self.sty, fy, gy, stp, fm, gm)
            self.fx, self.gx = fx + self.stx * gt, gx + gt
            self.fy, self.gy = fy + self.sty * gt, gy + gt
        else:
            (self.stx, self.fx, self.gx, self.sty, self.fy, self.gy, nstp) = self._interpolate(
                self.stx, self.fx, self.gx, self.sty, self.fy, self.gy, stp, f, g)
        if self.bracketed:
            if abs(self.sty - self.stx) >= 0.66 * self.width1:
                nstp = self.stx + 0.5 * (self.sty - self.stx)
            self.width1 = self.width
            self.width = abs(self.sty - self.stx)
            self.stmin, self.stmax = min(self.stx, self.sty), max(self.stx, self.sty)
        else:
            self.stmin = nstp + self.XTRAPL * (nstp - self.stx)
            self.stmax = nstp + self.XTRAPU * (nstp - self.stx)
        nstp = min(max(nstp, self.stpmin), self.stpmax)
        if (self.bracketed and (nstp <= self.stmin or nstp >= self.stmax)) or \
                (self.bracketed and self.stmax - self.stmin <= self.xtol * self.stmax):
            nstp = self.stx
        self.stp = nstp
        return "fg"

    def _interpolate(self, stx, fx, dx, sty, fy, dy, stp, fp, dp):
        """One safeguarded step of the interval update: the four cases of the method
        (higher value; derivative sign change; smaller derivative magnitude; otherwise),
        each choosing between the cubic and quadratic (secant) minimisers."""
        stpmin, stpmax = self.stmin, self.stmax
        sgnd = dp * math.copysign(1.0, dx)

        def cubic(a, fa, da, b, fb, db):
            # minimiser of the cubic through (a, fa, da), (b, fb, db), measured from b
            theta = 3.0 * (fa - fb) / (b - a) + da + db
            s = max(abs(theta), abs(da), abs(db))
            disc = (theta / s) ** 2 - (da / s) * (db / s)
            return theta, s, disc

        if fp > fx:
            theta, s, disc = cubic(stx, fx, dx, stp, fp, dp)
            gamma = s * math.sqrt(disc)
            if stp < stx:
                gamma = -gamma
            p = (gamma - dx) + theta
            q = ((gamma - dx) + gamma) + dp
            stpc = stx + (p / q) * (stp - stx)
            stpq = stx + ((dx / ((fx - fp) / (stp - stx) + dx)) / 2.0) * (stp - stx)
            stpf = stpc if abs(stpc - stx) < abs(stpq - stx) else stpc + (stpq - stpc) / 2.0
            self.bracketed = True
        elif sgnd < 0.0:
            theta, s, disc = cubic(stx, fx, dx, stp, fp, dp)
            gamma = s * math.sqrt(disc)
            if stp > stx:
                gamma = -gamma
            p = (gamma - dp) + theta
            q = ((gamma - dp) + gamma) + dx
            stpc = stp + (p / q) * (stx - stp)
            stpq = stp + (dp / (dp - dx)) * (stx - stp)
            stpf = stpc if abs(stpc - stp) > abs(stpq - stp) else stpq
            self.bracketed = True
        elif abs(dp) < abs(dx):
            theta, s, disc = cubic(stx, fx, dx, stp, fp, dp)
            gamma = s * math.sqrt(max(0.0, disc))
            if stp > stx:
                gamma = -gamma
            p = (gamma - dp) + theta
            q = (gamma + (dx - dp)) + gamma
            r = p / q
            if r < 0.0 and gamma != 0.0:
                stpc = stp + r * (stx - stp)
            elif stp > stx:
                stpc = stpmax
            else:
                stpc = stpmin
            stpq = stp + (dp / (dp - dx)) * (stx - stp)
            if self.bracketed:
                stpf = stpc if abs(stpc - stp) < abs(stpq - stp) else stpq
                if stp > stx:
                    stpf = min(stp + 0.66 * (sty - stp), stpf)
                else:
                    stpf = max(stp + 0.66 * (sty - stp), stpf)
            else:
                stpf = stpc if abs(stpc - stp) > abs(stpq - stp) else stpq
                stpf = min(max(stpf, stpmin), stpmax)
        else:
            if self.bracketed:
                theta, s, disc = cubic(sty, fy, dy, stp, fp, dp)
                gamma = s * math.sqrt(disc)
                if stp > sty:
                    gamma = -gamma
                p = (gamma - dp) + theta
                q = ((gamma - dp) + gamma) + dy
                stpf = stp + (p / q) * (sty - stp)
            elif stp > stx:
                stpf = stpmax
            else:
                stpf = stpmin
        if fp > fx:
            sty, fy, dy = stp, fp, dp
        else:
            if sgnd < 0.0:
                sty, fy, dy = stx, fx, dx
            stx, fx, dx = stp, fp, dp
        return stx, fx, dx, sty, fy, dy, stpf


def max_feasible_step(x, d, lower, big=1e10):
    """Largest step along d keeping x + stp d >= lower (big when d never decreases a
    variable); at least 1, since xbar = x + d is feasible."""
    neg = d < 0
    stp = big
    if neg.any():
        stp = min(big, float(np.min((lower[neg] - x[neg]) / d[neg])))
    return max(stp, 1.0)


def subspace_direction(x, xc, g, theta, W, M, c, free):
    """Unconstrained minimiser step du of the quadratic model over the free variables
    from xc (direct primal method, compact form)."""
    Wz = W[free]
    r = g[free] + theta * (xc[free] - x[free]) - Wz @ (M @ c)
    v = M @ (Wz.T @ r)
    N = np.eye(W.shape[1]) - (M @ (Wz.T @ Wz)) / theta
    u = np.linalg.solve(N, v)
    return -r / theta - (Wz @ u) / theta ** 2


# --------------------------------------------------------------------- command line
def lbfgsb(fun, x0, lower=None, m=10, maxiter=15000, maxfun=15000, ftol=2.2204460492503131e-09,
           gtol=1e-5, maxls=20, target=None):
    """Minimise fun (x -> (f, g)) subject to x >= lower.  Returns a dict with x, f, nit,
    nfev, message and the per-iteration history of (x, f)."""
    x = np.asarray(x0, dtype=np.float64).copy()
    n = x.size
    lower = np.full(n, 0.0) if lower is None else np.broadcast_to(np.asarray(lower, dtype=np.float64), (n,)).copy()
    x = np.maximum(x, lower)
    f, g = fun(x)
    nfev = 1
    hist = [(x.copy(), f)]
    S = np.zeros((n, 0))
    Y = np.zeros((n, 0))
    theta = 1.0
    it = 0
    msg = ""

    def done(reason):
        return {"x": x, "f": f, "nit": it, "nfev": nfev, "message": reason, "history": hist}

    if target is not None and f <= target:
        return done("target")
    if projected_gradient_norm(x, g, lower) <= gtol:
        return done("pgtol")
    while True:
        W = np.hstack([Y, theta * S])
        M = middle_matrix(S, Y, theta)
        xc, c, free = cauchy_point(x, g, lower, theta, W, M)
        xbar = subspace_step(x, xc, g, lower, theta, W, M, c, free)
        d = xbar - x
        gd = float(g @ d)
        ok = gd < 0.0
        if ok:
            if it == 0:
                stpmax = 1.0
                stp = min(1.0 / float(np.linalg.norm(d)), stpmax)
            else:
                stpmax = max_feasible_step(x, d, lower)
                stp = 1.0
            ls = MoreThuente(stpmin=0.0, stpmax=stpmax)
            ls.start(f, gd, stp)
            x_old, f_old, g_old = x, f, g
            evals = 0
            status = "fg"
            while True:
                xt = xbar.copy() if ls.stp == 1.0 else x_old + ls.stp * d
                ft, gt = fun(xt)
                nfev += 1
                evals += 1
                if target is not None and ft <= target:
                    x, f, g = xt, ft, gt
                    hist.append((x.copy(), f))
                    return done("target")
                status = ls.step(ft, float(gt @ d))
                if status in ("conv", "warn"):
                    break
                if evals >= maxls or nfev >= maxfun:
                    status = "fail"
                    break
            ok = status != "fail"
        if not ok:
            # discard the memory and retry from the last accepted iterate
            if S.shape[1] == 0:
                return done("abnormal termination in line search")
            S = np.zeros((n, 0))
            Y = np.zeros((n, 0))
            theta = 1.0
            if not gd < 0.0:
                continue
            x, f, g = x_old, f_old, g_old
            continue
        x, f, g = xt, ft, gt
        it += 1
        hist.append((x.copy(), f))
        if projected_gradient_norm(x, g, lower) <= gtol:
            return done("pgtol")
        if (f_old - f) / max(abs(f_old), abs(f), 1.0) <= ftol:
            return done("ftol")
        if it >= maxiter:
            return done("maxiter")
        if nfev >= maxfun:
            return done("maxfun")
        s = x - x_old
        y = g - g_old
        sy = float(s @ y)
        if sy > EPS * (-float(g_old @ s)):
            if S.shape[1] == m:
                S, Y = S[:, 1:], Y[:, 1:]
            S = np.hstack([S, s[:, None]])
            Y = np.hstack([Y, y[:, None]])
            theta = float(y @ y) / sy
