"""Positivity-bounded quasi-Newton loop around the GPU objective (Sect. 3.4,
Eq. L-BFGS-B).

`solve`: scipy's L-BFGS-B on the host in FP64 with bounds I >= 0, one HIP
objective+gradient evaluation per function call; x (H2D) and the gradient (D2H) cross
PCIe every evaluation.

`DeviceSolver`: the same method run on the GPU (include/ivx_lbfgsb.h), with the iterate,
gradient and correction pairs in device memory; only a few scalars per step reach the
host."""
from __future__ import annotations

import ctypes
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


# ----------------------------------------------------------------------- device loop
class _LbOptions(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("maxiter", ctypes.c_int32), ("maxfun", ctypes.c_int32),
                ("maxls", ctypes.c_int32), ("positivity", ctypes.c_int32), ("full_sort", ctypes.c_int32),
                ("stream_wait", ctypes.c_int32), ("reserved", ctypes.c_int32), ("ftol", ctypes.c_double), ("gtol", ctypes.c_double), ("target", ctypes.c_double)]


class _LbResult(ctypes.Structure):
    _fields_ = [("f", ctypes.c_double), ("pg_norm", ctypes.c_double), ("nit", ctypes.c_int64),
                ("nfev", ctypes.c_int64), ("reason", ctypes.c_int32), ("n_walks_full", ctypes.c_int32),
                ("n_walks", ctypes.c_int64)]


REASONS = {0: "pgtol", 1: "ftol", 2: "maxiter", 3: "maxfun", 4: "target", 5: "abnormal"}


def _lb_lib(plan):
    lib = plan.lib
    if getattr(lib, "_lb_ready", False):
        return lib
    vp = ctypes.c_void_p
    lib.ivx_lbfgsb_create.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(vp)]
    lib.ivx_lbfgsb_destroy.argtypes = [vp]
    lib.ivx_lbfgsb_default_options.argtypes = [ctypes.POINTER(_LbOptions)]
    lib.ivx_lbfgsb_solve.argtypes = [vp, vp, ctypes.POINTER(_LbOptions), vp, vp, ctypes.c_int64,
                                     ctypes.POINTER(_LbResult), vp]
    for f in ("ivx_lbfgsb_create", "ivx_lbfgsb_destroy", "ivx_lbfgsb_default_options", "ivx_lbfgsb_solve"):
        getattr(lib, f).restype = ctypes.c_int
    lib._lb_ready = True
    return lib


class DeviceSolver:
    """The bounded L-BFGS-B loop on the GPU (include/ivx_lbfgsb.h): FP64 iterate, gradient
    and memory in device memory, one ivx_objective_grad per evaluation, no host copies of
    the sky."""

    def __init__(self, plan, m_max: int = 10):
        self.plan = plan
        self.lib = _lb_lib(plan)
        h = ctypes.c_void_p()
        self._check(self.lib.ivx_lbfgsb_create(plan._h, int(m_max), ctypes.byref(h)))
        self._h = h

    def _check(self, code):
        if code != 0:
            from . import IvxError

            raise IvxError(code, self.lib.ivx_last_error().decode())

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.ivx_lbfgsb_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, x0=None, maxiter=15000, m=10, ftol=2.2204460492503131e-09, gtol=1e-5, maxls=20,
              maxfun=15000, target=None, positivity=True, history=20000, stream=None, t_start=None,
              full_sort=False, stream_wait=False):
        """Minimise Q_tot from x0 (None: zeros; numpy or cuda tensor).  Returns a SolveResult
        whose x is a cuda tensor [C][N][N] in the plan's precision.  full_sort: every Cauchy
        search sorts all breakpoints (the default sorts a sampled prefix first; the iterates
        are the same).  stream_wait: the host reads each step's results after the stream has
        drained instead of spinning on the flag the step publishes (the same iterates)."""
        import torch

        plan = self.plan
        shape = (plan.n_chan, plan.n_sky, plan.n_sky)
        if x0 is None:
            x = torch.zeros(shape, dtype=plan.torch_dtype, device="cuda")
        elif isinstance(x0, np.ndarray):
            x = torch.tensor(x0.reshape(shape), dtype=plan.torch_dtype, device="cuda")
        else:
            x = x0.reshape(shape).to(device="cuda", dtype=plan.torch_dtype).clone().contiguous()
        o = _LbOptions()
        self._check(self.lib.ivx_lbfgsb_default_options(ctypes.byref(o)))
        o.m, o.maxiter, o.maxfun, o.maxls = int(m), int(maxiter), int(maxfun), int(maxls)
        o.positivity = 1 if positivity else 0
        o.full_sort = 1 if full_sort else 0
        o.stream_wait = 1 if stream_wait else 0
        o.ftol, o.gtol = float(ftol), float(gtol)
        o.target = float(target) if target is not None else float("-inf")
        fh = np.zeros(max(int(history), 0), dtype=np.float64)
        th = np.zeros_like(fh)
        r = _LbResult()
        st = None if stream is None else stream.cuda_stream
        if st is None:
            st = torch.cuda.current_stream().cuda_stream
        t0 = time.perf_counter() if t_start is None else t_start
        t_call = time.perf_counter()
        self._check(self.lib.ivx_lbfgsb_solve(self._h, x.data_ptr(), ctypes.byref(o),
                                              fh.ctypes.data if fh.size else None,
                                              th.ctypes.data if fh.size else None, fh.size, ctypes.byref(r), st))
        offset = t_call - t0
        k = min(int(r.nfev), fh.size)
        hist = [(float(th[i]) + offset, float(fh[i])) for i in range(k)]
        res = SolveResult(x=x, fun=float(r.f), nfev=int(r.nfev), nit=int(r.nit), message=REASONS.get(r.reason, "?"),
                          seconds=time.perf_counter() - t0, history=hist, reached_target=(r.reason == 4))
        res.pg_norm = float(r.pg_norm)
        res.n_walks = int(r.n_walks)
        res.n_walks_full = int(r.n_walks_full)
        return res
