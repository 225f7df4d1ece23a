"""Python binding of libivx (the gfx950 Classic3D objective/gradient engine).

Argument marshalling only: every step of an evaluation runs in the HIP kernels behind the
C ABI declared in include/ivx.h.  PyTorch supplies device memory and the current stream.
There is no CPU fallback: if the shared library is missing the import of a Plan fails.

    from paper_2609_17636_amd import Plan, Objective, solve
    plan = Plan.from_problem(problem)          # geometry + hyper-parameters
    plan.set_problem_data(problem)             # visibilities, weights, beams, grids, SD map
    terms, grad = plan.objective_grad(sky)     # sky: cuda tensor [C][N][N]
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

from .build import lib_path

__all__ = ["Plan", "Objective", "ForwardModel", "solve", "DeviceSolver", "UNet", "load_library", "IvxError", "STATUS", "STAGES"]

STATUS = {0: "IVX_OK", -1: "IVX_EINVAL", -2: "IVX_ENOMEM", -3: "IVX_EHIP", -4: "IVX_ENONFINITE",
          -5: "IVX_ESTATE"}


class IvxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class _Problem(ctypes.Structure):
    _fields_ = [
        ("n_chan", ctypes.c_int32), ("n_sky", ctypes.c_int32), ("pixel_rad", ctypes.c_double),
        ("n_point", ctypes.c_int32), ("n_sub", ctypes.c_int32),
        ("vis_offsets", ctypes.POINTER(ctypes.c_int64)), ("flux_scale", ctypes.POINTER(ctypes.c_double)),
        ("lambda_r", ctypes.c_double), ("lambda_s", ctypes.c_double),
        ("sd_n", ctypes.c_int32), ("sd_stride", ctypes.c_int32), ("sd_offset", ctypes.c_int32),
        ("sd_fwhm_rad", ctypes.c_double), ("sd_sigma", ctypes.c_double), ("nufft_eps", ctypes.c_double),
        ("kernel_width", ctypes.c_int32), ("fine_size", ctypes.c_int32), ("tile", ctypes.c_int32),
        ("reserved", ctypes.c_int32), ("lambda_nu", ctypes.c_double),
    ]


EXPORTS = ("ivx_plan_create", "ivx_plan_set_data", "ivx_objective_grad", "ivx_forward", "ivx_adjoint",
           "ivx_autotune", "ivx_plan_info", "ivx_plan_destroy", "ivx_last_error", "ivx_version",
           "ivx_real_size", "ivx_set_timing", "ivx_stage_times", "ivx_set_graph", "ivx_set_blocking",
           "ivx_plan_set_vis", "ivx_set_gridder_occupancy", "ivx_set_fused_fold", "ivx_objective",
           "ivx_objective_forward", "ivx_objective_backward", "ivx_forward_adjoint", "ivx_last_terms",
           "ivx_nufft_probe", "ivx_plan_set_w", "ivx_plan_w_info", "ivx_sort_u64")

STAGES = ("image_rows", "col_fwd", "grid", "fold", "col_inv", "row_inv", "sd", "sky", "final")

_LIBS = {}


def load_library(precision: str = "f32") -> ctypes.CDLL:
    """Load libivx.so ("f32") or libivx_f64.so ("f64") from the package directory."""
    if precision in _LIBS:
        return _LIBS[precision]
    path = lib_path(precision)
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run __graft_entry__.build() or "
                           f"python -m paper_2609_17636_amd.build")
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.ivx_plan_create.argtypes = [ctypes.POINTER(_Problem), ctypes.POINTER(vp)]
    lib.ivx_plan_set_data.argtypes = [vp] * 9
    lib.ivx_plan_set_data_shared.argtypes = [vp] * 10
    lib.ivx_objective_grad.argtypes = [vp, vp, vp, vp, vp]
    lib.ivx_forward.argtypes = [vp, vp, vp, vp]
    lib.ivx_adjoint.argtypes = [vp, vp, vp, vp]
    lib.ivx_autotune.argtypes = [vp, dbl, vp, vp]
    lib.ivx_plan_info.argtypes = [vp, vp]
    lib.ivx_plan_destroy.argtypes = [vp]
    lib.ivx_set_timing.argtypes = [vp, ctypes.c_uint32]
    lib.ivx_set_graph.argtypes = [vp, ctypes.c_int]
    lib.ivx_set_blocking.argtypes = [vp, i32, i32, i32, i32, i32, vp]
    lib.ivx_plan_set_vis.argtypes = [vp, vp, vp, vp]
    lib.ivx_set_gridder_occupancy.argtypes = [vp, i32]
    lib.ivx_set_fused_fold.argtypes = [vp, ctypes.c_int]
    lib.ivx_objective.argtypes = [vp, vp, vp, vp]
    lib.ivx_objective_forward.argtypes = [vp, vp, vp, vp]
    lib.ivx_objective_backward.argtypes = [vp, vp, vp, dbl, vp]
    lib.ivx_forward_adjoint.argtypes = [vp, vp, vp, vp]
    lib.ivx_last_terms.argtypes = [vp, vp, vp]
    lib.ivx_nufft_probe.argtypes = [i32, i32, i32, vp]
    lib.ivx_plan_set_w.argtypes = [vp, vp, i32, dbl, vp]
    lib.ivx_plan_w_info.argtypes = [vp, vp]
    lib.ivx_sort_u64.argtypes = [vp, vp, vp, vp, i64, i32, vp]
    lib.ivx_sort_u64.restype = ctypes.c_int
    lib.ivx_stage_times.argtypes = [vp, vp, vp]
    lib.ivx_last_error.restype = ctypes.c_char_p
    lib.ivx_last_error.argtypes = []
    for f in ("ivx_plan_create", "ivx_plan_set_data", "ivx_objective_grad", "ivx_forward",
              "ivx_adjoint", "ivx_autotune", "ivx_plan_info", "ivx_plan_destroy", "ivx_set_timing",
              "ivx_stage_times", "ivx_set_graph", "ivx_set_blocking", "ivx_plan_set_vis",
              "ivx_set_gridder_occupancy", "ivx_set_fused_fold", "ivx_objective", "ivx_objective_forward",
              "ivx_objective_backward", "ivx_forward_adjoint", "ivx_last_terms", "ivx_nufft_probe"):
        getattr(lib, f).restype = ctypes.c_int
    lib.ivx_version.restype = ctypes.c_int
    lib.ivx_real_size.restype = ctypes.c_int
    _LIBS[precision] = lib
    return lib


def _torch():
    import torch

    return torch


def _ptr(a) -> Optional[int]:
    """Raw address of a numpy array or torch tensor (must be contiguous), or None."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        assert a.flags["C_CONTIGUOUS"]
        return a.ctypes.data
    assert a.is_contiguous()
    return a.data_ptr()


def _flags(f):
    if isinstance(f, np.ndarray):
        return np.ascontiguousarray(f, dtype=np.uint8)
    torch = _torch()
    return f.to(torch.uint8).contiguous()


def _stream_ptr(stream=None) -> Optional[int]:
    torch = _torch()
    if not torch.cuda.is_available():
        return None
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def nufft_probe(n_sub: int, n_fine: int, kernel_width: int, precision: str = "f32") -> float:
    """ivx_nufft_probe: worst one-dimensional error of a unit point source's transform."""
    lib = load_library(precision)
    e = np.zeros(1)
    code = lib.ivx_nufft_probe(int(n_sub), int(n_fine), int(kernel_width), e.ctypes.data)
    if code != 0:
        raise IvxError(code, lib.ivx_last_error().decode())
    return float(e[0])


def sort_u64(keys, values=None, end_bit: int = 64, precision: str = "f32"):
    """ivx_sort_u64: stable radix sort of a cuda int64 tensor (bit patterns taken as unsigned)
    on bits [0, end_bit), optionally carrying a cuda int32 tensor.  Returns (keys, values)."""
    torch = _torch()
    lib = load_library(precision)
    assert keys.is_cuda and keys.dtype == torch.int64 and keys.dim() == 1
    keys = keys.contiguous()
    out_k = torch.empty_like(keys)
    out_v = None
    if values is not None:
        assert values.is_cuda and values.dtype == torch.int32 and values.shape == keys.shape
        values = values.contiguous()
        out_v = torch.empty_like(values)
    code = lib.ivx_sort_u64(_ptr(keys), _ptr(out_k), _ptr(values), _ptr(out_v), keys.numel(), int(end_bit),
                            _stream_ptr())
    if code != 0:
        raise IvxError(code, lib.ivx_last_error().decode())
    return out_k, out_v


class Plan:
    """One Classic3D problem on the current GPU (see include/ivx.h for every argument)."""

    def __init__(self, n_chan, n_sky, pixel_rad, n_point, n_sub, vis_offsets, flux_scale,
                 lambda_r=0.0, lambda_s=0.0, sd_n=0, sd_stride=0, sd_offset=0, sd_fwhm_rad=0.0,
                 sd_sigma=0.0, precision="f32", nufft_eps=0.0, kernel_width=0, fine_size=0, tile=0, lambda_nu=0.0):
        self.lib = load_library(precision)
        self.precision = precision
        self.np_real = np.float32 if precision == "f32" else np.float64
        self.n_chan, self.n_sky, self.n_point, self.n_sub = int(n_chan), int(n_sky), int(n_point), int(n_sub)
        self._offsets = np.ascontiguousarray(vis_offsets, dtype=np.int64)
        self._fscale = np.ascontiguousarray(flux_scale, dtype=np.float64)
        self.n_vis = int(self._offsets[-1])
        self.lambda_r, self.lambda_s = float(lambda_r), float(lambda_s)
        d = _Problem()
        d.n_chan, d.n_sky, d.pixel_rad = self.n_chan, self.n_sky, float(pixel_rad)
        d.n_point, d.n_sub = self.n_point, self.n_sub
        d.vis_offsets = self._offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        d.flux_scale = self._fscale.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.lambda_r, d.lambda_s = float(lambda_r), float(lambda_s)
        d.sd_n, d.sd_stride, d.sd_offset = int(sd_n), int(sd_stride), int(sd_offset)
        d.sd_fwhm_rad, d.sd_sigma, d.nufft_eps = float(sd_fwhm_rad), float(sd_sigma), float(nufft_eps)
        d.kernel_width, d.fine_size, d.tile, d.reserved = int(kernel_width), int(fine_size), int(tile), 0
        d.lambda_nu = float(lambda_nu)
        self.lambda_nu = float(lambda_nu)
        h = ctypes.c_void_p()
        self._check(self.lib.ivx_plan_create(ctypes.byref(d), ctypes.byref(h)))
        self._h = h

    @classmethod
    def from_problem(cls, p, **kw):
        sd_on = p.sd_n > 0 and p.lambda_s != 0.0
        return cls(p.n_chan, p.n_sky, p.pixel_rad, p.n_point, p.n_sub, p.vis_offsets, p.flux_scale,
                   lambda_r=p.lambda_r, lambda_s=p.lambda_s if sd_on else 0.0,
                   sd_n=p.sd_n if sd_on else 0, sd_stride=p.sd_stride if sd_on else 0,
                   sd_offset=p.sd_offset if sd_on else 0, sd_fwhm_rad=p.sd_fwhm_rad if sd_on else 0.0,
                   sd_sigma=p.sd_sigma if sd_on else 0.0, lambda_nu=float(getattr(p, "lambda_nu", 0.0)), **kw)

    # -------------------------------------------------------------------- plumbing
    def _check(self, code):
        if code != 0:
            raise IvxError(code, self.lib.ivx_last_error().decode())

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.ivx_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _real(self, a):
        if a is None:
            return None
        if isinstance(a, np.ndarray):
            return np.ascontiguousarray(a, dtype=self.np_real)
        torch = _torch()
        return a.to(torch.float32 if self.precision == "f32" else torch.float64).contiguous()

    @property
    def torch_dtype(self):
        torch = _torch()
        return torch.float32 if self.precision == "f32" else torch.float64

    # ----------------------------------------------------------------------- data
    def _pairs(self, vis):
        """Complex numpy visibilities as a [M][2] real array (a view when the precision
        matches, so large host arrays are not copied)."""
        if isinstance(vis, np.ndarray) and np.iscomplexobj(vis):
            want = np.complex64 if self.precision == "f32" else np.complex128
            if vis.dtype == want and vis.flags.c_contiguous:
                return vis.view(self.np_real).reshape(-1, 2)
            return np.stack([vis.real, vis.imag], axis=-1)
        return vis

    def set_data(self, uv, vis, weight, beams, interp, flags=None, sd_map=None, stream=None):
        """uv [M][2], vis [M] complex or [M][2], weight [M], beams [P][n][n], interp
        [P][n][n][2], flags [M] uint8 or None, sd_map [C][sd][sd] or None (host numpy or
        cuda tensors)."""
        keep = [self._real(uv), self._real(self._pairs(vis)), self._real(weight), self._real(beams),
                self._real(interp), self._real(sd_map)]
        fl = None if flags is None else _flags(flags)
        uv_, vis_, w_, b_, g_, sd_ = keep
        self._check(self.lib.ivx_plan_set_data(self._h, _ptr(uv_), _ptr(vis_), _ptr(w_), _ptr(fl),
                                                _ptr(b_), _ptr(g_), _ptr(sd_), _stream_ptr(stream)))

    def set_data_shared(self, uv, weight, uv_scale, vis, beams, interp, flags=None, sd_map=None, stream=None):
        """Spectral cube with one uv track per pointing: uv [sum_k M_k][2] and weight
        [sum_k M_k] in pointing order, uv_scale [C] (channel c sees uv * uv_scale[c]),
        vis [M] complex or [M][2] and flags [M] per (pointing, channel) block."""
        keep = [self._real(uv), self._real(weight), self._real(self._pairs(vis)), self._real(beams),
                self._real(interp), self._real(sd_map)]
        sc = np.ascontiguousarray(uv_scale, dtype=np.float64)
        fl = None if flags is None else _flags(flags)
        uv_, w_, vis_, b_, g_, sd_ = keep
        self._check(self.lib.ivx_plan_set_data_shared(self._h, _ptr(uv_), _ptr(w_), sc.ctypes.data, _ptr(vis_),
                                                       _ptr(fl), _ptr(b_), _ptr(g_), _ptr(sd_),
                                                       _stream_ptr(stream)))

    def set_w(self, w, w_width: int = 0, w_sigma: float = 0.0, stream=None):
        """The full forward model of Eq. vis (1/n factor and w phase): w [M] (or [sum_k M_k] for
        a shared-uv plan) in wavelengths, caller order; None returns to the coplanar model."""
        w_ = self._real(w)
        self._check(self.lib.ivx_plan_set_w(self._h, _ptr(w_), int(w_width), float(w_sigma), _stream_ptr(stream)))

    def w_info(self) -> dict:
        a = np.zeros(6, dtype=np.float64)
        self._check(self.lib.ivx_plan_w_info(self._h, a.ctypes.data))
        return {"enabled": bool(a[0]), "planes": int(a[1]), "dw": float(a[2]), "x_centre": float(a[3]),
                "w_width": int(a[4]), "w_sigma": float(a[5])}

    def set_vis(self, vis, weight=None, stream=None):
        """New data (and weights) for the same observation: cuda tensors [M][2] (or complex
        numpy) and [M], caller order."""
        torch = _torch()
        if isinstance(vis, np.ndarray):
            if np.iscomplexobj(vis):
                vis = np.stack([vis.real, vis.imag], axis=-1)
            vis = torch.tensor(vis, dtype=self.torch_dtype, device="cuda")
        if isinstance(weight, np.ndarray):
            weight = torch.tensor(weight, dtype=self.torch_dtype, device="cuda")
        v = vis.to(self.torch_dtype).contiguous()
        w = None if weight is None else weight.to(self.torch_dtype).contiguous()
        self._check(self.lib.ivx_plan_set_vis(self._h, _ptr(v), _ptr(w), _stream_ptr(stream)))

    def set_cube_data(self, p, stream=None):
        """Data of a shared-uv spectral cube (synth.CubeProblem layout)."""
        sd = p.sd_map if (p.sd_n > 0 and p.lambda_s != 0.0) else None
        self.set_data_shared(p.uv, p.weight, p.uv_scale, p.vis, p.beams, p.interp, flags=p.flags, sd_map=sd,
                             stream=stream)

    def set_problem_data(self, p, stream=None):
        sd = p.sd_map if (p.sd_n > 0 and p.lambda_s != 0.0) else None
        self.set_data(p.uv, p.vis, p.weight, p.beams, p.interp, flags=p.flags, sd_map=sd, stream=stream)

    # ------------------------------------------------------------------ evaluation
    def objective_grad(self, sky, grad=None, terms=None, stream=None):
        """One evaluation at `sky` (cuda tensor [C][N][N]); returns (terms, grad) where terms
        is a host float64 array {Q_tot, Q, K, R} (or the given device tensor)."""
        torch = _torch()
        sky = sky.to(self.torch_dtype).contiguous()
        if grad is None:
            grad = torch.empty_like(sky)
        host_terms = terms is None
        if host_terms:
            terms = np.zeros(4, dtype=np.float64)
        self._check(self.lib.ivx_objective_grad(self._h, _ptr(sky), _ptr(grad), _ptr(terms),
                                                _stream_ptr(stream)))
        return terms, grad

    def objective(self, sky, terms=None, stream=None):
        """Q_tot terms {Q_tot, Q, K, R} only (no gradient work); host float64 array or the given
        device tensor."""
        sky = sky.to(self.torch_dtype).contiguous()
        if terms is None:
            terms = np.zeros(4, dtype=np.float64)
        self._check(self.lib.ivx_objective(self._h, _ptr(sky), _ptr(terms), _stream_ptr(stream)))
        return terms

    def objective_forward(self, sky, terms=None, stream=None):
        """First half of a reverse-mode evaluation (see ivx_objective_forward): the terms, with
        the plan holding what objective_backward needs.  `sky` must stay alive and unchanged
        until that call."""
        assert sky.dtype == self.torch_dtype and sky.is_contiguous()
        if terms is None:
            terms = np.zeros(4, dtype=np.float64)
        self._check(self.lib.ivx_objective_forward(self._h, _ptr(sky), _ptr(terms), _stream_ptr(stream)))
        return terms

    def objective_backward(self, sky, grad=None, scale=1.0, stream=None):
        """Second half: scale * dQ_tot/dx at the sky of the preceding objective_forward."""
        torch = _torch()
        if grad is None:
            grad = torch.empty_like(sky)
        self._check(self.lib.ivx_objective_backward(self._h, _ptr(sky), _ptr(grad), float(scale),
                                                    _stream_ptr(stream)))
        return grad

    def forward_adjoint(self, vis, out=None, stream=None):
        """Unweighted transpose of forward: Re sum_k P_k^T s A_k F^H vis, cuda tensor [C][N][N]."""
        torch = _torch()
        vis = vis.to(self.torch_dtype).contiguous()
        if out is None:
            out = torch.empty((self.n_chan, self.n_sky, self.n_sky), dtype=self.torch_dtype, device=vis.device)
        self._check(self.lib.ivx_forward_adjoint(self._h, _ptr(vis), _ptr(out), _stream_ptr(stream)))
        return out

    def forward(self, sky, out=None, stream=None):
        """Model visibilities in caller order, cuda tensor [M][2] (flagged entries 0)."""
        torch = _torch()
        sky = sky.to(self.torch_dtype).contiguous()
        if out is None:
            out = torch.empty((self.n_vis, 2), dtype=self.torch_dtype, device=sky.device)
        self._check(self.lib.ivx_forward(self._h, _ptr(sky), _ptr(out), _stream_ptr(stream)))
        return out

    def adjoint(self, vis, out=None, stream=None):
        """Re sum_k P_k^T s A_k F^H W vis, cuda tensor [C][N][N]."""
        torch = _torch()
        vis = vis.to(self.torch_dtype).contiguous()
        if out is None:
            out = torch.empty((self.n_chan, self.n_sky, self.n_sky), dtype=self.torch_dtype, device=vis.device)
        self._check(self.lib.ivx_adjoint(self._h, _ptr(vis), _ptr(out), _stream_ptr(stream)))
        return out

    def autotune(self, budget_ms=2000.0, stream=None) -> int:
        t = ctypes.c_int32(0)
        self._check(self.lib.ivx_autotune(self._h, float(budget_ms), ctypes.addressof(t), _stream_ptr(stream)))
        return int(t.value)

    def set_blocking(self, tile, waves, chunk, lanes, vpi, stream=None):
        """Explicit gridding blocking (see ivx_set_blocking); accuracy-neutral."""
        self._check(self.lib.ivx_set_blocking(self._h, int(tile), int(waves), int(chunk), int(lanes), int(vpi),
                                              _stream_ptr(stream)))

    def set_gridder_occupancy(self, waves_per_simd: int):
        """Matrix-core gridder build: 6 or 7 waves per SIMD, 0 = by work-item count."""
        self._check(self.lib.ivx_set_gridder_occupancy(self._h, int(waves_per_simd)))

    def set_fused_fold(self, mode: int):
        """Sum the gridding windows inside the inverse column pass: 1 where it pays (default),
        2 wherever the grid allows, 0 never (through the extended grid); results are
        identical."""
        self._check(self.lib.ivx_set_fused_fold(self._h, int(mode)))

    def set_graph(self, enable: bool):
        """Replay objective evaluations from a captured HIP graph (default) or launch eagerly."""
        self._check(self.lib.ivx_set_graph(self._h, int(bool(enable))))

    def set_timing(self, stages=STAGES):
        """Record device events around the named stages of every objective evaluation."""
        mask = 0
        for st in stages:
            mask |= 1 << STAGES.index(st)
        self._check(self.lib.ivx_set_timing(self._h, mask))

    def stage_times(self) -> tuple:
        """({stage: summed ms}, number of timed evaluations) since the last call."""
        ms = np.zeros(len(STAGES))
        n = np.zeros(1, dtype=np.int64)
        self._check(self.lib.ivx_stage_times(self._h, ms.ctypes.data, n.ctypes.data))
        return dict(zip(STAGES, ms.tolist())), int(n[0])

    def last_terms(self, stream=None) -> np.ndarray:
        """{Q_tot, Q, K, R, R_nu} of the last evaluation (synchronises the stream)."""
        t = np.zeros(5, dtype=np.float64)
        self._check(self.lib.ivx_last_terms(self._h, t.ctypes.data, _stream_ptr(stream)))
        return t

    def info(self) -> dict:
        a = np.zeros(16, dtype=np.int64)
        self._check(self.lib.ivx_plan_info(self._h, a.ctypes.data))
        keys = ["n_fine", "kernel_width", "tile", "n_work_items", "n_live_vis", "n_slots", "device_bytes",
                "n_items", "ext_rows", "ext_cols", "graph_nodes", "window", "waves_per_block",
                "chunk", "lanes", "vpi"]
        return {k: int(v) for k, v in zip(keys, a)}


def _autograd_functions():
    torch = _torch()

    class Objective(torch.autograd.Function):
        """Q_tot(x) as a differentiable scalar (Eq. fusion_cost).  Forward: the value alone
        (ivx_objective) when x needs no gradient, else ivx_objective_forward, whose pass over
        the visibilities also spreads the weighted residuals.  Backward: the hand-written
        adjoint half, ivx_objective_backward, scaled by the incoming gradient (the paper gets
        this gradient by automatic differentiation, Sect. 3.4)."""

        @staticmethod
        def forward(ctx, x, plan):
            xs = x.detach().to(plan.torch_dtype).contiguous()
            if ctx.needs_input_grad[0]:
                terms = plan.objective_forward(xs)
                ctx.plan = plan
                ctx.in_dtype = x.dtype
                ctx.save_for_backward(xs)
            else:
                terms = plan.objective(xs)
            return torch.tensor(terms[0], dtype=torch.float64, device=x.device)

        @staticmethod
        def backward(ctx, gout):
            (xs,) = ctx.saved_tensors
            grad = ctx.plan.objective_backward(xs, scale=float(gout))
            return grad.to(ctx.in_dtype), None

    class ForwardModel(torch.autograd.Function):
        """Model visibilities V(x) [M][2] in the caller's order (ivx_forward, Sect. 2.1); the
        backward pass is the unweighted transpose ivx_forward_adjoint."""

        @staticmethod
        def forward(ctx, x, plan):
            ctx.plan = plan
            ctx.in_dtype = x.dtype
            return plan.forward(x.detach())

        @staticmethod
        def backward(ctx, g):
            return ctx.plan.forward_adjoint(g.contiguous()).to(ctx.in_dtype), None

    return {"Objective": Objective, "ForwardModel": ForwardModel}


_AUTOGRAD = {}


def __getattr__(name):
    if name in ("Objective", "ForwardModel"):
        if not _AUTOGRAD:
            _AUTOGRAD.update(_autograd_functions())
        return _AUTOGRAD[name]
    raise AttributeError(name)


from .solver import DeviceSolver, solve  # noqa: E402
from .unet import UNet  # noqa: E402
