"""Binding of include/ivx_dataproc.h: SIN interpolation and deprojection grids, beam
resampling, linear mosaicking and feathering on the GPU (argument marshalling only)."""
from __future__ import annotations

import ctypes

import numpy as np


class SinFrame(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("reserved", ctypes.c_int32), ("delta", ctypes.c_double),
                ("ra", ctypes.c_double), ("dec", ctypes.c_double)]


def _lib(precision="f32"):
    from . import load_library

    lib = load_library(precision)
    if getattr(lib, "_dp_ready", False):
        return lib
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    fp = ctypes.POINTER(SinFrame)
    lib.ivx_dp_sin_grids.argtypes = [fp, i32, vp, i32, dbl, vp, vp]
    lib.ivx_dp_deprojection_grids.argtypes = [fp, i32, vp, i32, dbl, vp, vp]
    lib.ivx_dp_resample_beams.argtypes = [i32, vp, i32, dbl, i32, dbl, vp, vp]
    lib.ivx_linear_mosaic.argtypes = [i32, i32, i32, vp, vp, i32, vp, dbl, vp, vp, vp]
    lib.ivx_feather_work_bytes.argtypes = [i32, i32]
    lib.ivx_feather_work_bytes.restype = ctypes.c_int64
    lib.ivx_feather.argtypes = [i32, i32, dbl, dbl, vp, vp, vp, vp, vp]
    for f in ("ivx_dp_sin_grids", "ivx_dp_deprojection_grids", "ivx_dp_resample_beams", "ivx_linear_mosaic",
              "ivx_feather"):
        getattr(lib, f).restype = ctypes.c_int
    lib._dp_ready = True
    return lib


def _check(lib, code):
    if code != 0:
        from . import IvxError

        raise IvxError(code, lib.ivx_last_error().decode())


def _torch():
    import torch

    return torch


def _dtype(precision):
    torch = _torch()
    return torch.float32 if precision == "f32" else torch.float64


def _stream():
    return _torch().cuda.current_stream().cuda_stream


def _centres(centres):
    c = np.ascontiguousarray(centres, dtype=np.float64).reshape(-1, 2)
    return c


def sin_grids(n_sky, sky_delta, ra0, dec0, centres, n_sub, sub_delta, precision="f32"):
    """[P][n_sub][n_sub][2] interpolation grids (cuda tensor); centres [P][2] (ra, dec)."""
    torch = _torch()
    lib = _lib(precision)
    c = _centres(centres)
    out = torch.empty((c.shape[0], n_sub, n_sub, 2), dtype=_dtype(precision), device="cuda")
    f = SinFrame(int(n_sky), 0, float(sky_delta), float(ra0), float(dec0))
    _check(lib, lib.ivx_dp_sin_grids(ctypes.byref(f), c.shape[0], c.ctypes.data, int(n_sub), float(sub_delta),
                                     out.data_ptr(), _stream()))
    return out


def deprojection_grids(n_sky, sky_delta, ra0, dec0, centres, n_sub, sub_delta, precision="f32"):
    """[P][n_sky][n_sky][2] sub-image positions of every sky pixel (cuda tensor)."""
    torch = _torch()
    lib = _lib(precision)
    c = _centres(centres)
    out = torch.empty((c.shape[0], n_sky, n_sky, 2), dtype=_dtype(precision), device="cuda")
    f = SinFrame(int(n_sky), 0, float(sky_delta), float(ra0), float(dec0))
    _check(lib, lib.ivx_dp_deprojection_grids(ctypes.byref(f), c.shape[0], c.ctypes.data, int(n_sub),
                                              float(sub_delta), out.data_ptr(), _stream()))
    return out


def resample_beams(beams_in, beam_delta, n_sub, sub_delta):
    """[P][nb][nb] beams of pixel size beam_delta -> [P][n_sub][n_sub] at sub_delta."""
    torch = _torch()
    precision = "f32" if beams_in.dtype == torch.float32 else "f64"
    lib = _lib(precision)
    b = beams_in.contiguous()
    out = torch.empty((b.shape[0], n_sub, n_sub), dtype=b.dtype, device=b.device)
    _check(lib, lib.ivx_dp_resample_beams(b.shape[0], b.data_ptr(), b.shape[1], float(beam_delta), int(n_sub),
                                          float(sub_delta), out.data_ptr(), _stream()))
    return out


def linear_mosaic(sub_images, beams, deproj, pb_min=0.0):
    """Eq. linear / Eq. pb_eff: (image [C][N][N], pb_eff [N][N]) from sub_images [P][C][n][n],
    beams [P][n][n] and deprojection grids [P][N][N][2] (cuda tensors of one precision)."""
    torch = _torch()
    precision = "f32" if sub_images.dtype == torch.float32 else "f64"
    lib = _lib(precision)
    s, b, d = sub_images.contiguous(), beams.contiguous(), deproj.contiguous()
    P, C, n = s.shape[0], s.shape[1], s.shape[2]
    N = d.shape[1]
    img = torch.empty((C, N, N), dtype=s.dtype, device=s.device)
    peff = torch.empty((N, N), dtype=s.dtype, device=s.device)
    _check(lib, lib.ivx_linear_mosaic(P, C, n, s.data_ptr(), b.data_ptr(), N, d.data_ptr(), float(pb_min),
                                      img.data_ptr(), peff.data_ptr(), _stream()))
    return img, peff


def feather(interf, single_dish, delta, theta, out=None):
    """App. B feathering of [C][n][n] maps (cuda tensors); returns the combined maps."""
    torch = _torch()
    precision = "f32" if interf.dtype == torch.float32 else "f64"
    lib = _lib(precision)
    a, s = interf.contiguous(), single_dish.contiguous()
    C, n = a.shape[0], a.shape[-1]
    nbytes = lib.ivx_feather_work_bytes(C, n)
    if nbytes < 0:
        raise ValueError("n must be a power of two in [64, 2048]")
    work = torch.empty(nbytes, dtype=torch.uint8, device=a.device)
    if out is None:
        out = torch.empty_like(a)
    _check(lib, lib.ivx_feather(C, n, float(delta), float(theta), a.data_ptr(), s.data_ptr(), out.data_ptr(),
                                work.data_ptr(), _stream()))
    return out


def bench(n_point_side: int = 6, n_sky: int = 1024, n_sub: int = 384, n_chan: int = 128, reps: int = 10) -> dict:
    """Device time of each data-processor and image-domain call at the spectral cube's
    geometry (36 pointings of 384^2 over a 1024^2 sky at 30 arcsec, 128 channels): grids,
    deprojection grids, beam resampling from 512^2 beam images, the linear mosaic of 36 x 128
    sub-images and the feathering of 128 maps.  Algorithmic bytes: each array read or written
    once (the bilinear taps of a sub-image and the gathers of the mosaic count their source
    once); the fraction is against the 8 TB/s HBM peak."""
    import time

    torch = _torch()
    arcsec = np.pi / (180.0 * 3600.0)
    delta = 30.0 * arcsec
    ra0, dec0 = 1.387, -1.2049
    pitch = 120.0 * delta
    c = n_point_side
    centres = np.array([[ra0 + ((j - (c - 1) / 2) * pitch + (0.5 * pitch if i % 2 else 0.0)) / np.cos(dec0),
                         dec0 + (i - (c - 1) / 2) * pitch * np.sqrt(3) / 2] for i in range(c) for j in range(c)])
    P = centres.shape[0]
    g = torch.Generator(device="cuda").manual_seed(0)
    nb = 512
    beams_in = torch.rand((P, nb, nb), generator=g, device="cuda")
    sub = torch.rand((P, n_chan, n_sub, n_sub), generator=g, device="cuda")
    maps = torch.rand((n_chan, n_sky, n_sky), generator=g, device="cuda")
    sd = torch.rand((n_chan, n_sky, n_sky), generator=g, device="cuda")
    out = {}

    def timed(name, fn, nbytes):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = fn()
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / reps
        gbs = nbytes / (ms * 1e-3) / 1e9
        out[name] = {"ms": ms, "algorithmic_bytes": float(nbytes), "achieved_gbs": gbs, "frac": gbs / 8000.0}
        return r

    grids = timed("sin_grids", lambda: sin_grids(n_sky, delta, ra0, dec0, centres, n_sub, delta), P * n_sub * n_sub * 8)
    dep = timed("deprojection_grids", lambda: deprojection_grids(n_sky, delta, ra0, dec0, centres, n_sub, delta),
                P * n_sky * n_sky * 8)
    beams = timed("resample_beams", lambda: resample_beams(beams_in, 20.0 * arcsec, n_sub, delta),
                  P * (nb * nb + n_sub * n_sub) * 4)
    timed("linear_mosaic", lambda: linear_mosaic(sub, beams, dep, 0.2),
          P * n_sky * n_sky * 8 + P * (n_chan + 1) * n_sub * n_sub * 4 + (n_chan + 1) * n_sky * n_sky * 4)
    timed("feather", lambda: feather(maps, sd, delta, 30.0 * 60.0 * arcsec),
          n_chan * n_sky * n_sky * (3 * 4 + 2 * 8))
    del grids
    out["geometry"] = {"n_point": P, "n_sky": n_sky, "n_sub": n_sub, "n_chan": n_chan, "beam_image": nb,
                       "reps": reps}
    return out


if __name__ == "__main__":
    import argparse
    import json

    ap = argparse.ArgumentParser(description="device time of the data-processor and image-domain calls")
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--n-chan", type=int, default=128)
    a = ap.parse_args()
    print(json.dumps(bench(n_chan=a.n_chan, reps=a.reps)), flush=True)
