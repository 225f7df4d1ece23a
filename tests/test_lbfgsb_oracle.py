"""Pins of the FP64 L-BFGS-B oracle (CPU): the Cauchy point against exhaustive piecewise
minimisation of the dense quadratic model, the subspace step against a dense solve, the
line search against the strong Wolfe conditions, and whole solves against scipy's
L-BFGS-B and against non-negative least squares."""
import numpy as np
import pytest
import scipy.optimize

from oracle import lbfgsb as L


def _state(seed, n=14, k=3):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    A = A @ A.T + n * np.eye(n)
    S = rng.standard_normal((n, k))
    Y = A @ S
    theta = float(Y[:, -1] @ Y[:, -1] / (S[:, -1] @ Y[:, -1]))
    x = np.maximum(rng.standard_normal(n), 0.0)
    x[:3] = 0.0
    g = rng.standard_normal(n)
    g[0] = abs(g[0])   # at the bound and pushed into it: fixed from the start
    g[1] = -abs(g[1])  # at the bound, moving away
    return x, g, np.zeros(n), S, Y, theta


def _path_minimiser(x, g, lower, B):
    """First local minimiser of m(z) = g.(z-x) + 1/2 (z-x).B(z-x) along z(t) = max(x - t g,
    lower), by walking the segments of the path with the dense B."""
    t_br = np.where(g > 0, (x - lower) / np.where(g > 0, g, 1.0), np.inf)
    ts = np.unique(np.concatenate([[0.0], t_br[np.isfinite(t_br)]]))
    ts = ts[ts >= 0]
    for j, t0 in enumerate(ts):
        t1 = ts[j + 1] if j + 1 < len(ts) else np.inf
        z0 = np.maximum(x - t0 * g, lower)
        d = np.where(t_br > t0, -g, 0.0)
        gm = g + B @ (z0 - x)          # model gradient at z0
        b = float(gm @ d)
        c = float(d @ B @ d)
        if b >= 0:
            return z0
        tau = -b / c if c > 0 else np.inf
        if tau < t1 - t0:
            return z0 + tau * d
    raise AssertionError("unbounded model")


@pytest.mark.parametrize("seed", range(6))
def test_cauchy_point_matches_exhaustive_path_search(seed):
    x, g, lower, S, Y, theta = _state(seed)
    W = np.hstack([Y, theta * S])
    M = L.middle_matrix(S, Y, theta)
    B = L.dense_B(S, Y, theta)
    xc, c, free = L.cauchy_point(x, g, lower, theta, W, M)
    np.testing.assert_allclose(xc, _path_minimiser(x, g, lower, B), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(c, W.T @ (xc - x), rtol=1e-10, atol=1e-12)
    assert not free[0] and np.all(xc[~free] == lower[~free])


def test_cauchy_point_with_empty_memory_is_projected_steepest_descent_minimiser():
    x, g, lower, _, _, _ = _state(7)
    W = np.zeros((x.size, 0))
    xc, _, _ = L.cauchy_point(x, g, lower, 1.0, W, np.zeros((0, 0)))
    np.testing.assert_allclose(xc, _path_minimiser(x, g, lower, np.eye(x.size)), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("seed", range(4))
def test_subspace_direction_is_the_dense_reduced_newton_step(seed):
    x, g, lower, S, Y, theta = _state(10 + seed)
    W = np.hstack([Y, theta * S])
    M = L.middle_matrix(S, Y, theta)
    B = L.dense_B(S, Y, theta)
    xc, c, free = L.cauchy_point(x, g, lower, theta, W, M)
    du = L.subspace_direction(x, xc, g, theta, W, M, c, free)
    rhs = -(g + B @ (xc - x))[free]
    np.testing.assert_allclose(du, np.linalg.solve(B[np.ix_(free, free)], rhs), rtol=1e-9, atol=1e-12)


def test_middle_matrix_reproduces_the_bfgs_matrix():
    """The compact form equals k explicit BFGS updates of theta I."""
    x, g, lower, S, Y, theta = _state(20)
    B = theta * np.eye(x.size)
    for i in range(S.shape[1]):
        s, y = S[:, i], Y[:, i]
        Bs = B @ s
        B = B - np.outer(Bs, Bs) / (s @ Bs) + np.outer(y, y) / (y @ s)
    np.testing.assert_allclose(L.dense_B(S, Y, theta), B, rtol=1e-10, atol=1e-10)


def test_line_search_satisfies_strong_wolfe():
    # phi(a) = f(x + a d) for a smooth 1-D function with a known minimiser region
    f = lambda a: (a - 3.0) ** 4 + 0.5 * a * a - 4 * a
    df = lambda a: 4 * (a - 3.0) ** 3 + a - 4
    for a0 in (1e-3, 1.0, 10.0):
        ls = L.MoreThuente(stpmax=1e3)
        ls.start(f(0.0), df(0.0), a0)
        for _ in range(30):
            st = ls.step(f(ls.stp), df(ls.stp))
            if st != "fg":
                break
        a = ls.stp
        assert st == "conv"
        assert f(a) <= f(0) + 1e-3 * a * df(0)
        assert abs(df(a)) <= 0.9 * abs(df(0))


def _nnls_case(seed, m=40, n=25):
    rng = np.random.default_rng(seed)
    C = rng.standard_normal((m, n))
    e = rng.standard_normal(m)
    fun = lambda x: (0.5 * float(np.sum((C @ x - e) ** 2)), C.T @ (C @ x - e))
    return C, e, fun


@pytest.mark.parametrize("seed", range(3))
def test_solution_of_nonnegative_least_squares(seed):
    C, e, fun = _nnls_case(seed)
    want, _ = scipy.optimize.nnls(C, e)
    r = L.lbfgsb(fun, np.zeros(C.shape[1]), gtol=1e-12, ftol=0.0, maxiter=2000)
    assert (want == 0).sum() >= 3       # the bounds bind
    np.testing.assert_allclose(r["x"], want, atol=1e-8)


@pytest.mark.parametrize("seed", range(3))
def test_iterates_follow_scipy_lbfgsb(seed):
    """Same method, same rules: the first iterates agree with scipy's L-BFGS-B to
    rounding, and both end at the same point."""
    C, e, fun = _nnls_case(seed)
    n = C.shape[1]
    xs = []
    res = scipy.optimize.minimize(fun, np.zeros(n), jac=True, method="L-BFGS-B",
                                  bounds=scipy.optimize.Bounds(np.zeros(n), np.full(n, np.inf)),
                                  options={"maxcor": 10, "gtol": 1e-12, "ftol": 0.0, "maxiter": 2000},
                                  callback=lambda xk: xs.append(np.array(xk)))
    r = L.lbfgsb(fun, np.zeros(n), gtol=1e-12, ftol=0.0, maxiter=2000)
    ours = [h[0] for h in r["history"][1:]]
    k = min(8, len(xs), len(ours))
    for i in range(k):
        np.testing.assert_allclose(ours[i], xs[i], rtol=1e-7, atol=1e-9, err_msg=f"iterate {i + 1}")
    np.testing.assert_allclose(r["x"], res.x, atol=1e-8)


def test_bounded_rosenbrock_matches_scipy():
    def fun(x):
        f = np.sum(100.0 * (x[1:] - x[:-1] ** 2) ** 2 + (1 - x[:-1]) ** 2)
        g = np.zeros_like(x)
        g[:-1] = -400 * x[:-1] * (x[1:] - x[:-1] ** 2) - 2 * (1 - x[:-1])
        g[1:] += 200 * (x[1:] - x[:-1] ** 2)
        return float(f), g
    lower = np.array([0.0, 0.0, 1.5, 0.0, 0.0, 0.0])
    x0 = np.full(6, 2.0)
    res = scipy.optimize.minimize(fun, x0, jac=True, method="L-BFGS-B",
                                  bounds=scipy.optimize.Bounds(lower, np.full(6, np.inf)),
                                  options={"gtol": 1e-10, "ftol": 0.0, "maxiter": 5000})
    r = L.lbfgsb(fun, x0, lower=lower, gtol=1e-10, ftol=0.0, maxiter=5000)
    np.testing.assert_allclose(r["x"], res.x, atol=1e-6)
    assert r["f"] == pytest.approx(res.fun, rel=1e-10, abs=1e-12)
