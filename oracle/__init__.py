"""FP64 CPU oracle of the Classic3D objective Q_tot and its gradient.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code with the
HIP path (no kernels, headers, tables or helpers); the two meet only through the seeded
inputs of the ``synth`` package.

Every function below is the plain definition of one step, evaluated with direct sums in
FP64, in the order of the paper:

  O1 reproject           sky -> SIN sub-image of pointing k by bilinear interpolation on
                         the precomputed grid (Sect. 2.1, Eq. sin_projection; Sect. 3.3)
  O2 beam                f = s * A_k * x'                              (Sect. 2.1)
  O3 dft_forward         direct non-uniform DFT, coplanar model        (Sect. 2.1)
     dft_forward_w       the full model of Eq. vis: the 1/n factor and the phase
                         w (n - 1) of every pixel, n = sqrt(1 - l^2 - m^2) (Sect. 2.1);
                         used for every block when the problem carries w
  O4 data term           r = V - y,  J_k = 1/2 sum w |r|^2,  w = 1/sigma^2
                                                                        (Sect. 2.2, Eq. Q)
  O5 dft_adjoint         explicit adjoint of O3 (real part)            (Sect. 3.4: the
                         gradient of Q_tot)
     dft_adjoint_w       explicit adjoint of dft_forward_w (real part)
  O6 reproject_adjoint   transpose of O1 (scatter of the bilinear weights)
  O7 regulariser         R = sum_c 1/2 ||D x_c||^2 with the 3x3 Laplacian d, zero padding;
                         grad = D (D x)                                  (Sect. 2.2, Eq. 3)
  O8 sd_term             T~ = S(B (x) x), K = 1/2 ||(T~ - T)/sigma_sd||^2,
                         grad = B^T S^T (T~ - T)/sigma_sd^2             (Sect. 2.4)
  O9 objective_grad      Q_tot = Q + lambda_s K + lambda_r R           (Eq. fusion_cost)
                         + lambda_nu R_nu, R_nu = 1/2 sum_c ||x_{c+1} - x_c||^2: a spectral
                         smoothness term coupling adjacent channels (one of the regulariser
                         extensions the paper names in Sect. 2.3 and its prospects; the form
                         is this repository's reading, the paper gives none)

The readings taken where the paper is silent (pixel <-> (l, m) mapping, bilinear
convention, boundary handling, single-dish sampling and normalisation, weights) are the
same ones the HIP path implements; they are listed with the design notes of the
repository.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build() -> str:
    """Compile the C part of the oracle (direct DFT and its adjoint) with gcc/OpenMP."""
    src = os.path.join(_HERE, "dft.c")
    tmp = _SO + ".tmp"
    subprocess.run(["gcc", "-O3", "-fPIC", "-shared", "-fopenmp", "-o", tmp, src, "-lm"],
                   check=True)
    os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.orc_dft_forward.argtypes = [ctypes.c_int, ctypes.c_double, dp, ctypes.c_int64, dp, dp]
        lib.orc_dft_forward.restype = None
        lib.orc_dft_adjoint.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int64, dp, dp, dp]
        lib.orc_dft_adjoint.restype = None
        lib.orc_dft_adjoint_pixels.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int64, dp, dp,
                                               ctypes.c_int64, ctypes.POINTER(ctypes.c_int32), dp]
        lib.orc_dft_adjoint_pixels.restype = None
        lib.orc_dft_forward_w.argtypes = [ctypes.c_int, ctypes.c_double, dp, ctypes.c_int64, dp, dp]
        lib.orc_dft_forward_w.restype = None
        lib.orc_dft_adjoint_w.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int64, dp, dp, dp]
        lib.orc_dft_adjoint_w.restype = None
        lib.orc_dft_adjoint_w_pixels.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int64, dp, dp,
                                                 ctypes.c_int64, ctypes.POINTER(ctypes.c_int32), dp]
        lib.orc_dft_adjoint_w_pixels.restype = None
        lib.orc_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def num_threads() -> int:
    return int(_load().orc_num_threads())


# ----------------------------------------------------------------------------- O3 / O5

def dft_forward(f: np.ndarray, uv: np.ndarray, delta: float) -> np.ndarray:
    """O3: V_j = sum_{a,b} f[a,b] exp(-2 pi i (u_j (b - n/2) + v_j (a - n/2)) delta)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    n = f.shape[0]
    assert f.shape == (n, n)
    uv = np.ascontiguousarray(uv, dtype=np.float64).reshape(-1, 2)
    out = np.empty((uv.shape[0], 2), dtype=np.float64)
    if uv.shape[0]:
        _load().orc_dft_forward(n, float(delta), _dp(f), uv.shape[0], _dp(uv), _dp(out))
    return out[:, 0] + 1j * out[:, 1]


def dft_adjoint(coef: np.ndarray, uv: np.ndarray, delta: float, n: int) -> np.ndarray:
    """O5: g[a,b] = Re sum_j c_j exp(+2 pi i (u_j (b - n/2) + v_j (a - n/2)) delta)."""
    coef = np.asarray(coef, dtype=np.complex128).ravel()
    cc = np.ascontiguousarray(np.stack([coef.real, coef.imag], axis=1))
    uv = np.ascontiguousarray(uv, dtype=np.float64).reshape(-1, 2)
    g = np.zeros((n, n), dtype=np.float64)
    if uv.shape[0]:
        _load().orc_dft_adjoint(int(n), float(delta), uv.shape[0], _dp(uv), _dp(cc), _dp(g))
    return g


def dft_adjoint_pixels(coef: np.ndarray, uv: np.ndarray, delta: float, n: int, pixels) -> np.ndarray:
    """O5 at selected pixels (a, b) only: one direct sum over all visibilities each."""
    coef = np.asarray(coef, dtype=np.complex128).ravel()
    cc = np.ascontiguousarray(np.stack([coef.real, coef.imag], axis=1))
    uv = np.ascontiguousarray(uv, dtype=np.float64).reshape(-1, 2)
    pix = np.ascontiguousarray(pixels, dtype=np.int32).reshape(-1, 2)
    out = np.zeros(pix.shape[0])
    if uv.shape[0] and pix.shape[0]:
        _load().orc_dft_adjoint_pixels(int(n), float(delta), uv.shape[0], _dp(uv), _dp(cc), pix.shape[0],
                                       pix.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(out))
    return out


def _check_uvw(uvw: np.ndarray, n: int, delta: float) -> np.ndarray:
    uvw = np.ascontiguousarray(uvw, dtype=np.float64).reshape(-1, 3)
    c = n // 2
    r2 = ((n - 1 - c) ** 2 + c ** 2) * float(delta) ** 2
    assert r2 < 1.0, "every pixel must lie inside the unit circle of direction cosines"
    return uvw


def dft_forward_w(f: np.ndarray, uvw: np.ndarray, delta: float) -> np.ndarray:
    """O3 with the w-term (Eq. vis): V_j = sum_{a,b} f[a,b] / n_ab
    exp(-2 pi i (u_j l_b + v_j m_a + w_j (n_ab - 1))), l_b = (b - n/2) delta,
    m_a = (a - n/2) delta, n_ab = sqrt(1 - l_b^2 - m_a^2)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    n = f.shape[0]
    assert f.shape == (n, n)
    uvw = _check_uvw(uvw, n, delta)
    out = np.empty((uvw.shape[0], 2), dtype=np.float64)
    if uvw.shape[0]:
        _load().orc_dft_forward_w(n, float(delta), _dp(f), uvw.shape[0], _dp(uvw), _dp(out))
    return out[:, 0] + 1j * out[:, 1]


def dft_adjoint_w(coef: np.ndarray, uvw: np.ndarray, delta: float, n: int) -> np.ndarray:
    """Adjoint of dft_forward_w on real images: g[a,b] = Re sum_j c_j / n_ab
    exp(+2 pi i (u_j l_b + v_j m_a + w_j (n_ab - 1)))."""
    coef = np.asarray(coef, dtype=np.complex128).ravel()
    cc = np.ascontiguousarray(np.stack([coef.real, coef.imag], axis=1))
    uvw = _check_uvw(uvw, n, delta)
    g = np.zeros((n, n), dtype=np.float64)
    if uvw.shape[0]:
        _load().orc_dft_adjoint_w(int(n), float(delta), uvw.shape[0], _dp(uvw), _dp(cc), _dp(g))
    return g


def dft_adjoint_w_pixels(coef: np.ndarray, uvw: np.ndarray, delta: float, n: int, pixels) -> np.ndarray:
    """dft_adjoint_w at selected pixels (a, b) only: one direct sum over all visibilities each."""
    coef = np.asarray(coef, dtype=np.complex128).ravel()
    cc = np.ascontiguousarray(np.stack([coef.real, coef.imag], axis=1))
    uvw = _check_uvw(uvw, n, delta)
    pix = np.ascontiguousarray(pixels, dtype=np.int32).reshape(-1, 2)
    out = np.zeros(pix.shape[0])
    if uvw.shape[0] and pix.shape[0]:
        _load().orc_dft_adjoint_w_pixels(int(n), float(delta), uvw.shape[0], _dp(uvw), _dp(cc), pix.shape[0],
                                         pix.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(out))
    return out


def block_forward(p, f: np.ndarray, s: slice, live: np.ndarray) -> np.ndarray:
    """Model visibilities of the live samples of block s: the full model (dft_forward_w)
    when the problem carries w coordinates, else the coplanar one (dft_forward)."""
    w = getattr(p, "w", None)
    if w is None:
        return dft_forward(f, p.uv[s][live], p.pixel_rad)
    uvw = np.concatenate([p.uv[s][live].astype(np.float64), w[s][live].astype(np.float64)[:, None]], axis=1)
    return dft_forward_w(f, uvw, p.pixel_rad)


def block_adjoint(p, coef: np.ndarray, s: slice, live: np.ndarray) -> np.ndarray:
    """Adjoint of block_forward for the live samples of block s (an n_sub^2 image)."""
    w = getattr(p, "w", None)
    if w is None:
        return dft_adjoint(coef, p.uv[s][live], p.pixel_rad, p.n_sub)
    uvw = np.concatenate([p.uv[s][live].astype(np.float64), w[s][live].astype(np.float64)[:, None]], axis=1)
    return dft_adjoint_w(coef, uvw, p.pixel_rad, p.n_sub)


# ----------------------------------------------------------------------------- O1 / O6

def _bilinear_taps(grid: np.ndarray, n_sky: int):
    """The four (row, col, weight) taps of every sub-pixel: i0 = floor(sy), j0 = floor(sx),
    weights (1-fy)(1-fx), (1-fy)fx, fy(1-fx), fy fx; taps outside the sky get weight 0."""
    sy = grid[..., 0].astype(np.float64)
    sx = grid[..., 1].astype(np.float64)
    i0 = np.floor(sy).astype(np.int64)
    j0 = np.floor(sx).astype(np.int64)
    fy = sy - i0
    fx = sx - j0
    taps = []
    for di, dj, w in ((0, 0, (1 - fy) * (1 - fx)), (0, 1, (1 - fy) * fx),
                      (1, 0, fy * (1 - fx)), (1, 1, fy * fx)):
        ii, jj = i0 + di, j0 + dj
        inside = (ii >= 0) & (ii < n_sky) & (jj >= 0) & (jj < n_sky)
        taps.append((np.where(inside, ii, 0), np.where(inside, jj, 0), np.where(inside, w, 0.0)))
    return taps


def reproject(sky: np.ndarray, grid: np.ndarray) -> np.ndarray:
    """O1: x'[a,b] = bilinear sample of the sky at grid[a,b] = (row, col); pixel (i, j)
    sits at coordinate (i, j); sky pixels outside [0, N)^2 contribute 0."""
    sky = np.asarray(sky, dtype=np.float64)
    out = np.zeros(grid.shape[:2])
    for ii, jj, w in _bilinear_taps(grid, sky.shape[0]):
        out += w * sky[ii, jj]
    return out


def reproject_adjoint(g: np.ndarray, grid: np.ndarray, n_sky: int) -> np.ndarray:
    """O6: transpose of O1: sky[i, j] += sum over sub-pixels of (weight of (i, j)) * g."""
    out = np.zeros(n_sky * n_sky)
    g = np.asarray(g, dtype=np.float64)
    for ii, jj, w in _bilinear_taps(grid, n_sky):
        out += np.bincount((ii * n_sky + jj).ravel(), weights=(w * g).ravel(),
                           minlength=n_sky * n_sky)
    return out.reshape(n_sky, n_sky)


# ----------------------------------------------------------------------------- O7

LAPLACIAN_KERNEL = np.array([[0.0, -1.0, 0.0], [-1.0, 4.0, -1.0], [0.0, -1.0, 0.0]])


def laplacian(x: np.ndarray) -> np.ndarray:
    """D x with the kernel d of Sect. 2.2 and zero padding ("same" size):
    (Dx)[i,j] = 4 x[i,j] - x[i-1,j] - x[i+1,j] - x[i,j-1] - x[i,j+1]."""
    x = np.asarray(x, dtype=np.float64)
    p = np.pad(x, 1)
    return 4.0 * x - p[:-2, 1:-1] - p[2:, 1:-1] - p[1:-1, :-2] - p[1:-1, 2:]


def regulariser(x: np.ndarray):
    """O7 for one channel: R = 1/2 ||D x||^2 and grad R = D^T D x = D (D x) (D is symmetric
    under zero padding)."""
    dx = laplacian(x)
    return 0.5 * float(np.sum(dx * dx)), laplacian(dx)


# ----------------------------------------------------------------------------- spectral term

def spectral_term(x: np.ndarray):
    """R_nu = 1/2 sum_{c=0}^{C-2} sum_r (x[c+1, r] - x[c, r])^2 over the cube [C][N][N] and its
    gradient: dR_nu/dx[c] = (x[c] - x[c-1]) [c >= 1] - (x[c+1] - x[c]) [c <= C-2]."""
    x = np.asarray(x, dtype=np.float64)
    g = np.zeros_like(x)
    val = 0.0
    for c in range(x.shape[0] - 1):
        d = x[c + 1] - x[c]
        val += 0.5 * float(np.sum(d * d))
        g[c] -= d
        g[c + 1] += d
    return val, g


# ----------------------------------------------------------------------------- O8

def sd_beam_taps(fwhm_rad: float, pixel_rad: float):
    """Unit-sum 1-D Gaussian taps g(t), |t| <= R_B = ceil(4 sigma_B / delta),
    sigma_B = FWHM / (2 sqrt(2 ln 2)).  Returns (taps[2 R_B + 1], R_B)."""
    sig = fwhm_rad / (2.0 * np.sqrt(2.0 * np.log(2.0)))
    rb = int(np.ceil(4.0 * sig / pixel_rad))
    t = np.arange(-rb, rb + 1, dtype=np.float64)
    g = np.exp(-(t * pixel_rad) ** 2 / (2.0 * sig * sig))
    return g / g.sum(), rb


def sd_sampling_matrix(n_sky: int, sd_n: int, stride: int, offset: int, taps, rb) -> np.ndarray:
    """G[p, i] = g(offset + p * stride - i): one axis of the separable beam, point-sampled
    at the single-dish pixel centres offset + p * stride (zero beyond R_B)."""
    G = np.zeros((sd_n, n_sky))
    for p in range(sd_n):
        centre = offset + p * stride
        for i in range(max(0, centre - rb), min(n_sky, centre + rb + 1)):
            G[p, i] = taps[i - centre + rb]
    return G


def sd_forward(x: np.ndarray, G: np.ndarray) -> np.ndarray:
    """T~[p, q] = sum_{i,j} g(o + pS - i) g(o + qS - j) x[i, j]  (beam, then sampling)."""
    return G @ np.asarray(x, dtype=np.float64) @ G.T


def sd_adjoint(e: np.ndarray, G: np.ndarray) -> np.ndarray:
    """Transpose of sd_forward: B^T S^T e."""
    return G.T @ np.asarray(e, dtype=np.float64) @ G


def sd_term(x: np.ndarray, t_map: np.ndarray, sigma: float, G: np.ndarray):
    """O8 for one channel: K = 1/2 sum ((T~ - T)/sigma)^2, grad = B^T S^T (T~ - T)/sigma^2."""
    res = sd_forward(x, G) - np.asarray(t_map, dtype=np.float64)
    return 0.5 * float(np.sum(res * res)) / sigma ** 2, sd_adjoint(res / sigma ** 2, G)


def sd_matrix_for(p) -> np.ndarray:
    taps, rb = sd_beam_taps(p.sd_fwhm_rad, p.pixel_rad)
    return sd_sampling_matrix(p.n_sky, p.sd_n, p.sd_stride, p.sd_offset, taps, rb)


# ----------------------------------------------------------------------------- blocks

def _live(p, s: slice):
    if p.flags is None:
        return np.ones(s.stop - s.start, dtype=bool)
    return p.flags[s] == 0


def beam_weighted_subimage(p, x_c: np.ndarray, k: int, c: int) -> np.ndarray:
    """O1 + O2: f = s_c * A_k * reproject(x_c, grid_k)."""
    return p.flux_scale[c] * p.beams[k].astype(np.float64) * reproject(x_c, p.interp[k])


def model_vis(p, x: np.ndarray) -> np.ndarray:
    """Model visibilities of every (pointing, channel) block, caller order; flagged
    entries are 0."""
    out = np.zeros(p.n_vis, dtype=np.complex128)
    x = np.asarray(x, dtype=np.float64).reshape(p.n_chan, p.n_sky, p.n_sky)
    for k in range(p.n_point):
        for c in range(p.n_chan):
            s = p.block(k, c)
            if s.stop == s.start:
                continue
            live = _live(p, s)
            f = beam_weighted_subimage(p, x[c], k, c)
            v = np.zeros(s.stop - s.start, dtype=np.complex128)
            v[live] = block_forward(p, f, s, live)
            out[s] = v
    return out


def adjoint_image(p, vis: np.ndarray, weighted: bool = True) -> np.ndarray:
    """Re sum_k P_k^T s A_k F^H W v over every block (flagged entries skipped):
    the transpose of model_vis with the natural weights."""
    vis = np.asarray(vis, dtype=np.complex128)
    g = np.zeros((p.n_chan, p.n_sky, p.n_sky))
    for k in range(p.n_point):
        for c in range(p.n_chan):
            s = p.block(k, c)
            if s.stop == s.start:
                continue
            live = _live(p, s)
            coef = vis[s][live] * (p.weight[s][live].astype(np.float64) if weighted else 1.0)
            gk = block_adjoint(p, coef, s, live)
            gk *= p.flux_scale[c] * p.beams[k].astype(np.float64)
            g[c] += reproject_adjoint(gk, p.interp[k], p.n_sky)
    return g


def objective_grad(p, x: np.ndarray):
    """O1-O9: returns ({"Q_tot", "Q", "K", "R"}, grad [C][N][N]) in FP64."""
    x = np.asarray(x, dtype=np.float64).reshape(p.n_chan, p.n_sky, p.n_sky)
    grad = np.zeros_like(x)
    Q = 0.0
    for k in range(p.n_point):
        for c in range(p.n_chan):
            s = p.block(k, c)
            if s.stop == s.start:
                continue
            live = _live(p, s)
            y = p.vis[s][live].astype(np.complex128)
            w = p.weight[s][live].astype(np.float64)
            f = beam_weighted_subimage(p, x[c], k, c)            # O1, O2
            r = block_forward(p, f, s, live) - y                  # O3, O4
            Q += 0.5 * float(np.sum(w * (r.real ** 2 + r.imag ** 2)))
            gk = block_adjoint(p, w * r, s, live)                 # O5
            gk *= p.flux_scale[c] * p.beams[k].astype(np.float64)
            grad[c] += reproject_adjoint(gk, p.interp[k], p.n_sky)  # O6
    R = 0.0
    K = 0.0
    G = sd_matrix_for(p) if (p.lambda_s != 0.0 and p.sd_map is not None and p.sd_n) else None
    for c in range(p.n_chan):
        if p.lambda_r != 0.0:
            rc, gr = regulariser(x[c])                             # O7
            R += rc
            grad[c] += p.lambda_r * gr
        if G is not None:
            kc, gk = sd_term(x[c], p.sd_map[c], p.sd_sigma, G)     # O8
            K += kc
            grad[c] += p.lambda_s * gk
    lam_nu = float(getattr(p, "lambda_nu", 0.0))
    Nu = 0.0
    if lam_nu != 0.0:
        Nu, gnu = spectral_term(x)
        grad += lam_nu * gnu
    terms = {"Q": Q, "K": K, "R": R, "Nu": Nu,
             "Q_tot": Q + p.lambda_s * K + p.lambda_r * R + lam_nu * Nu}  # O9
    return terms, grad


def sd_model(p, x: np.ndarray) -> np.ndarray:
    """Single-dish model T~ of every channel (used to synthesise the single-dish map)."""
    G = sd_matrix_for(p)
    x = np.asarray(x, dtype=np.float64).reshape(p.n_chan, p.n_sky, p.n_sky)
    return np.stack([sd_forward(x[c], G) for c in range(p.n_chan)])


def synthesize(p, with_sd: bool = True):
    """Attach oracle-generated data to a synth problem: y = model(x_true) + noise and,
    if the problem has a single-dish geometry, T = sd_model(x_true) + noise."""
    from synth import attach_data, attach_sd

    attach_data(p, model_vis(p, p.x_true))
    if with_sd and p.sd_n:
        attach_sd(p, sd_model(p, p.x_true))
    return p
