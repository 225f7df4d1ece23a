"""Positivity-bounded quasi-Newton loop around the GPU objective (Sect. 3.4,
Eq. L-BFGS-B): scipy's L-BFGS-B on the host in FP64 with bounds I >= 0, one HIP
objective+gradient evaluation per function call.  Only x (H2D) and the gradient (D2H)
cross PCIe; the evaluation itself is one call into libivx."""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np


class _Reached(Exception):
    pass


@dataclass
class SolveResult:
    x: np.ndarray
    fun: float
    nfev: int
    nit: int
    message: str
    seconds: float
    history: list = field(default_factory=list)  # (seconds since start, Q_tot) per evaluation
    reached_target: bool = False


def solve(plan, x0=None, maxiter=500, m=10, ftol=2.2e-9, gtol=1e-5, maxls=20, target=None,
          positivity=True, stream=None, t_start=None) -> SolveResult:
    """Minimise Q_tot with L-BFGS-B from x0 (zeros: the null prior).  With `target`, stop at
    the first evaluation whose Q_tot <= target (time-to-tolerance).  `t_start` lets a caller
    include work done before the solve (e.g. a warm start) in the history clock."""
    import scipy.optimize
    import torch

    C, N = plan.n_chan, plan.n_sky
    n = C * N * N
    x0 = np.zeros(n) if x0 is None else np.asarray(x0, dtype=np.float64).reshape(-1).copy()
    if positivity:
        np.maximum(x0, 0.0, out=x0)
    dev = torch.device("cuda")
    sky = torch.empty(n, dtype=plan.torch_dtype, device=dev)
    grad = torch.empty(n, dtype=plan.torch_dtype, device=dev)
    host = torch.empty(n, dtype=plan.torch_dtype, pin_memory=True)
    hist = []
    t0 = time.perf_counter() if t_start is None else t_start
    best = {"f": np.inf, "x": x0.copy()}

    def fun(x):
        host.numpy()[:] = x
        sky.copy_(host, non_blocking=False)
        terms, _ = plan.objective_grad(sky.view(C, N, N), grad=grad.view(C, N, N), stream=stream)
        g = grad.cpu().numpy().astype(np.float64)
        f = float(terms[0])
        hist.append((time.perf_counter() - t0, f))
        if f < best["f"]:
            best["f"], best["x"] = f, x.copy()
        if target is not None and f <= target:
            raise _Reached
        return f, g

    bounds = scipy.optimize.Bounds(np.zeros(n), np.full(n, np.inf)) if positivity else None
    reached = False
    try:
        r = scipy.optimize.minimize(fun, x0, jac=True, method="L-BFGS-B", bounds=bounds,
                                    options={"maxiter": maxiter, "maxcor": m, "ftol": ftol,
                                             "gtol": gtol, "maxls": maxls})
        x, f, nfev, nit, msg = r.x, float(r.fun), int(r.nfev), int(r.nit), str(r.message)
    except _Reached:
        reached = True
        x, f, nfev, nit, msg = best["x"], best["f"], len(hist), -1, "target reached"
    return SolveResult(x=x.reshape(C, N, N), fun=f, nfev=nfev, nit=nit, message=msg,
                       seconds=time.perf_counter() - t0, history=hist, reached_target=reached)
