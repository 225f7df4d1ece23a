"""Seeded synthetic inputs for the Classic3D objective (sky cubes, uv tracks, beams,
interpolation grids, flags, noise, single-dish geometry).

This module only *draws inputs*: it holds none of the arithmetic of the method itself
(no Fourier transform, no reprojection, no regulariser).  Model visibilities are
computed by whoever consumes a problem (the FP64 oracle in tests, the HIP path in the
benchmark) and attached with :func:`attach_data`, which only adds the drawn noise.

Every concern draws from its own sub-stream of ``numpy.random.SeedSequence(seed)``
(layout, field, tracks, flags, noise, sources) so that changing one size does not
reshuffle the others.

Geometry follows the paper's setting: a 36-antenna array observing with Earth-rotation
synthesis (Sect. 4, 5), Gaussian primary beams of 1 degree FWHM (Sect. 4.4), an
orthographic (SIN) sub-image per pointing reached by bilinear interpolation on a
precomputed grid (Sect. 2.1, Eq. sin_projection; Sect. 3.3), and a Gaussian
single-dish beam of 16 arcmin (Sect. 4.4).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

ARCSEC = np.pi / (180.0 * 3600.0)
ARCMIN = 60.0 * ARCSEC
DEG = np.pi / 180.0
C_LIGHT = 299_792_458.0
K_BOLTZMANN = 1.380649e-23
JY = 1e-26

# LMC centre used for the paper's simulations (Sect. 4.2, 4.4): 05h17m36s, -69d02m.
LMC_RA = (5.0 + 17.0 / 60.0 + 36.0 / 3600.0) * 15.0 * DEG
LMC_DEC = -(69.0 + 2.0 / 60.0) * DEG
ASKAP_LAT = -26.7 * DEG


@dataclass
class Problem:
    """One objective: sky cube [C][N][N], P pointings with n_sub x n_sub sub-images,
    visibilities stored block-wise, block index = k * n_chan + c (pointing-major)."""

    name: str
    n_chan: int
    n_sky: int
    pixel_rad: float
    n_point: int
    n_sub: int
    flux_scale: np.ndarray  # [C] float64, Jy per pixel per sky unit
    lambda_r: float
    lambda_s: float
    uv: np.ndarray  # [M, 2] float32, wavelengths
    vis_offsets: np.ndarray  # [P*C + 1] int64
    weight: np.ndarray  # [M] float32 (1 / sigma^2)
    flags: Optional[np.ndarray]  # [M] uint8, 1 = flagged, or None
    beams: np.ndarray  # [P][n_sub][n_sub] float32, peak 1
    interp: np.ndarray  # [P][n_sub][n_sub][2] float32, (row, col) sky coordinates
    x_true: np.ndarray  # [C][N][N] float64
    noise: np.ndarray  # [M] complex128, unit variance per component
    noise_rule: tuple  # ("abs", sigma) or ("frac_peak", fraction)
    sd_n: int = 0
    sd_stride: int = 0
    sd_offset: int = 0
    sd_fwhm_rad: float = 0.0
    sd_sigma: float = 0.0
    sd_map: Optional[np.ndarray] = None  # [C][sd_n][sd_n] float32
    sd_noise_frac: float = 0.01
    vis: Optional[np.ndarray] = None  # [M] complex64, filled by attach_data
    lambda_nu: float = 0.0  # spectral smoothness weight (couples adjacent channels)
    meta: dict = field(default_factory=dict)
    w: Optional[np.ndarray] = None  # [M] float32, wavelengths; None: the coplanar model

    @property
    def n_vis(self) -> int:
        return int(self.vis_offsets[-1])

    @property
    def n_items(self) -> int:
        return self.n_point * self.n_chan

    def block(self, k: int, c: int) -> slice:
        i = k * self.n_chan + c
        return slice(int(self.vis_offsets[i]), int(self.vis_offsets[i + 1]))


# ----------------------------------------------------------------------------- streams

def _streams(seed: int, names):
    ss = np.random.SeedSequence(seed)
    kids = ss.spawn(len(names))
    return {n: np.random.Generator(np.random.PCG64(s)) for n, s in zip(names, kids)}


_STREAMS = ("layout", "field", "tracks", "flags", "noise", "sources", "extra")


# ----------------------------------------------------------------------------- array

def antenna_layout(rng, n_ant: int = 36, radius_m: float = 3000.0) -> np.ndarray:
    """East/North antenna positions [n_ant][2] uniform in a disk (max baseline <= 2R)."""
    r = radius_m * np.sqrt(rng.uniform(0.0, 1.0, n_ant))
    th = rng.uniform(0.0, 2.0 * np.pi, n_ant)
    return np.stack([r * np.cos(th), r * np.sin(th)], axis=1)


def baselines(enu: np.ndarray) -> np.ndarray:
    """All i<j antenna differences [n_bl][2] (East, North), metres."""
    i, j = np.triu_indices(enu.shape[0], k=1)
    return enu[j] - enu[i]


def uvw_tracks(bl_en: np.ndarray, n_time: int, dec: float, freq_hz: float,
               lat: float = ASKAP_LAT, ha_hours: float = 6.0) -> np.ndarray:
    """Earth-rotation synthesis tracks (textbook ENU -> XYZ -> uvw rotation), time-major:
    returns [n_time * n_bl][3] (u, v, w) in wavelengths, hour angle uniform over
    [-ha/2, +ha/2]."""
    east, north = bl_en[:, 0], bl_en[:, 1]
    X = -np.sin(lat) * north
    Y = east
    Z = np.cos(lat) * north
    ha = np.linspace(-0.5, 0.5, n_time) * ha_hours * (2.0 * np.pi / 24.0)
    sH, cH = np.sin(ha)[:, None], np.cos(ha)[:, None]
    u = sH * X[None, :] + cH * Y[None, :]
    v = -np.sin(dec) * cH * X[None, :] + np.sin(dec) * sH * Y[None, :] + np.cos(dec) * Z[None, :]
    w = np.cos(dec) * cH * X[None, :] - np.cos(dec) * sH * Y[None, :] + np.sin(dec) * Z[None, :]
    lam = C_LIGHT / freq_hz
    return np.stack([u.ravel(), v.ravel(), w.ravel()], axis=1) / lam


def uv_tracks(bl_en: np.ndarray, n_time: int, dec: float, freq_hz: float,
              lat: float = ASKAP_LAT, ha_hours: float = 6.0) -> np.ndarray:
    """The (u, v) columns of :func:`uvw_tracks` (the coplanar model of Sect. 2.1 uses no w)."""
    return np.ascontiguousarray(uvw_tracks(bl_en, n_time, dec, freq_hz, lat, ha_hours)[:, :2])


# ----------------------------------------------------------------------------- skies

def grf_k3(rng, n: int, slope: float = 3.0) -> np.ndarray:
    """Periodic Gaussian random field with P(k) ~ k^-slope, zero mean, unit variance."""
    ky = np.fft.fftfreq(n)[:, None]
    kx = np.fft.rfftfreq(n)[None, :]
    kk = np.sqrt(kx * kx + ky * ky)
    amp = np.zeros_like(kk)
    amp[kk > 0] = kk[kk > 0] ** (-slope / 2.0)
    white = rng.standard_normal((n, n))
    g = np.fft.irfft2(np.fft.rfft2(white) * amp, s=(n, n))
    g -= g.mean()
    return g / g.std()


def lognormal_field(g: np.ndarray, peak: float = 50.0) -> np.ndarray:
    """exp of a Gaussian field, min-max scaled to [0, peak] (positive diffuse sky)."""
    e = np.exp(g)
    return peak * (e - e.min()) / (e.max() - e.min())


def ar1_cube(rng, n_chan: int, n: int, rho: float = 0.9, peak: float = 50.0) -> np.ndarray:
    """Channel-correlated log-normal cube: g_c = rho g_{c-1} + sqrt(1-rho^2) eps_c,
    exp, cube-global min-max to [0, peak]."""
    g = np.empty((n_chan, n, n))
    g[0] = grf_k3(rng, n)
    s = np.sqrt(1.0 - rho * rho)
    for c in range(1, n_chan):
        g[c] = rho * g[c - 1] + s * grf_k3(rng, n)
    e = np.exp(g)
    return peak * (e - e.min()) / (e.max() - e.min())


def rj_flux_scale(freq_hz: float, pixel_rad: float) -> float:
    """Rayleigh-Jeans K -> Jy per pixel: 2 k_B nu^2 / c^2 * Omega_pix / 1e-26 (App. B)."""
    return 2.0 * K_BOLTZMANN * freq_hz ** 2 / C_LIGHT ** 2 * pixel_rad ** 2 / JY


# ----------------------------------------------------------------------------- beams

def gaussian_pb(n_sub: int, pixel_rad: float, fwhm_rad: float) -> np.ndarray:
    """Primary beam A(l, m) = exp(-4 ln2 (l^2+m^2)/FWHM^2), peak 1 at sub-pixel
    (n_sub/2, n_sub/2); l along columns, m along rows."""
    t = (np.arange(n_sub) - n_sub // 2) * pixel_rad
    r2 = t[:, None] ** 2 + t[None, :] ** 2
    return np.exp(-4.0 * np.log(2.0) * r2 / fwhm_rad ** 2)


def identity_interp(n_sub: int, row0: float = 0.0, col0: float = 0.0) -> np.ndarray:
    """Interpolation grid of an integer (or constant) translation: sub-pixel (a, b)
    samples sky coordinate (row0 + a, col0 + b)."""
    a = np.arange(n_sub, dtype=np.float64)
    g = np.empty((n_sub, n_sub, 2))
    g[..., 0] = row0 + a[:, None]
    g[..., 1] = col0 + a[None, :]
    return g


def _sin_fwd(ra, dec, ra0, dec0):
    """Orthographic (SIN) direction cosines of (ra, dec) about (ra0, dec0)."""
    l = np.cos(dec) * np.sin(ra - ra0)
    m = np.sin(dec) * np.cos(dec0) - np.cos(dec) * np.sin(dec0) * np.cos(ra - ra0)
    return l, m


def _sin_inv(l, m, ra0, dec0):
    n = np.sqrt(np.maximum(0.0, 1.0 - l * l - m * m))
    dec = np.arcsin(m * np.cos(dec0) + n * np.sin(dec0))
    ra = ra0 + np.arctan2(l, n * np.cos(dec0) - m * np.sin(dec0))
    return ra, dec


def sin_interp(n_sky: int, n_sub: int, pixel_rad: float, centre_rowcol, ra0=LMC_RA, dec0=LMC_DEC):
    """Interpolation grid of one pointing (Sect. 3.3): for every sub-pixel (a, b) of a SIN
    sub-image centred on sky pixel ``centre_rowcol`` (both frames share the pixel size),
    the (row, col) position of the same sky direction in the mosaic's SIN frame centred
    on (ra0, dec0) at pixel (n_sky/2, n_sky/2).  Returns the grid and the pointing
    centre (ra, dec)."""
    pr, pc = centre_rowcol
    lk = (pc - n_sky / 2) * pixel_rad
    mk = (pr - n_sky / 2) * pixel_rad
    rak, deck = _sin_inv(lk, mk, ra0, dec0)
    t = (np.arange(n_sub) - n_sub // 2) * pixel_rad
    L, M = np.meshgrid(t, t)  # L varies along columns, M along rows
    ra, dec = _sin_inv(L, M, rak, deck)
    l, m = _sin_fwd(ra, dec, ra0, dec0)
    g = np.empty((n_sub, n_sub, 2))
    g[..., 0] = m / pixel_rad + n_sky / 2
    g[..., 1] = l / pixel_rad + n_sky / 2
    return g, (float(rak), float(deck))


def hex_centres(n_rows: int, n_cols: int, pitch_px: float, n_sky: int) -> np.ndarray:
    """Close-packed hexagonal footprint (Sect. 4.4): rows spaced pitch*sqrt(3)/2, odd
    rows offset by half a pitch, centred on the sky.  Returns [P][2] (row, col)."""
    dy = pitch_px * np.sqrt(3.0) / 2.0
    pts = []
    for r in range(n_rows):
        for c in range(n_cols):
            pts.append((r * dy, c * pitch_px + (0.5 * pitch_px if r % 2 else 0.0)))
    pts = np.array(pts)
    pts -= pts.mean(axis=0)
    return pts + n_sky / 2


# ----------------------------------------------------------------------------- data

def attach_data(p: Problem, model_vis: np.ndarray) -> Problem:
    """y = model + sigma * noise, with natural weights 1/sigma^2.  The noise rule is
    ("abs", sigma) or ("frac_peak", f): sigma = f * max |model| of each block."""
    model_vis = np.asarray(model_vis, dtype=np.complex128)
    y = np.empty(p.n_vis, dtype=np.complex128)
    w = np.empty(p.n_vis, dtype=np.float32)
    kind, val = p.noise_rule
    for i in range(p.n_items):
        s = slice(int(p.vis_offsets[i]), int(p.vis_offsets[i + 1]))
        if s.stop == s.start:
            continue
        if kind == "abs":
            sig = val
        else:
            live = model_vis[s] if p.flags is None else model_vis[s][p.flags[s] == 0]
            peak = np.abs(live).max() if live.size else 1.0
            sig = val * (peak if peak > 0 else 1.0)
        y[s] = model_vis[s] + sig * p.noise[s]
        w[s] = 1.0 / (sig * sig)
    p.vis = y.astype(np.complex64)
    p.weight = w
    return p


def attach_sd(p: Problem, sd_model: np.ndarray) -> Problem:
    """Single-dish map T = model + noise, sigma_sd = frac * max T (per channel, Sect. 2.4)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(p.meta.get("seed", 0) + 17)))
    t = np.asarray(sd_model, dtype=np.float64)
    sig = p.sd_noise_frac * float(np.abs(t).max() if t.size else 1.0)
    p.sd_sigma = sig if sig > 0 else 1.0
    p.sd_map = (t + p.sd_sigma * rng.standard_normal(t.shape)).astype(np.float32)
    return p


def attach_sd_level(p, level: float = 25.0):
    """Single-dish map for timing runs that need no meaningful fusion residual: a constant
    level plus 1% noise per pixel, sigma_sd = 1% of the level.  (Tests synthesise the map
    from the sky instead; the cost of the evaluation does not depend on these values.)"""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(p.meta.get("seed", 0) + 19)))
    shape = (p.n_chan, p.sd_n, p.sd_n)
    p.sd_sigma = p.sd_noise_frac * level
    p.sd_map = (level + p.sd_sigma * rng.standard_normal(shape)).astype(np.float32)
    return p


# ----------------------------------------------------------------------------- configs

def single_pointing(name: str, seed: int, n_sky: int, pixel_arcsec: float, n_time: int,
                    n_keep: Optional[int], sky: str, lambda_r: float, noise_rule,
                    freq_hz: float = 1.4e9, fwhm_deg: float = 1.0, flag_rate: float = 0.0,
                    n_ant: int = 36, radius_m: float = 3000.0, n_src: int = 5, w_term: bool = False) -> Problem:
    """One pointing, one channel, identity interpolation grid (sub-image = sky); w_term:
    the problem carries the w coordinate of every sample (the full model of Eq. vis)."""
    st = _streams(seed, _STREAMS)
    pix = pixel_arcsec * ARCSEC
    enu = antenna_layout(st["layout"], n_ant, radius_m)
    uvw = uvw_tracks(baselines(enu), n_time, LMC_DEC, freq_hz)
    if n_keep is not None:
        uvw = uvw[:n_keep]
    uv = np.ascontiguousarray(uvw[:, :2])
    m = uv.shape[0]
    if sky == "points":
        x = np.zeros((1, n_sky, n_sky))
        lo, hi = n_sky // 8, n_sky - n_sky // 8
        cells = st["sources"].choice((hi - lo) ** 2, size=n_src, replace=False)
        flux = st["sources"].uniform(0.1, 1.0, n_src)
        for cidx, f in zip(cells, flux):
            x[0, lo + cidx // (hi - lo), lo + cidx % (hi - lo)] = f
        scale = 1.0
    else:
        x = lognormal_field(grf_k3(st["field"], n_sky))[None]
        scale = rj_flux_scale(freq_hz, pix)
    flags = None
    if flag_rate > 0:
        flags = (st["flags"].uniform(size=m) < flag_rate).astype(np.uint8)
    noise = st["noise"].standard_normal(m) + 1j * st["noise"].standard_normal(m)
    return Problem(
        name=name, n_chan=1, n_sky=n_sky, pixel_rad=pix, n_point=1, n_sub=n_sky,
        flux_scale=np.array([scale]), lambda_r=lambda_r, lambda_s=0.0,
        uv=uv.astype(np.float32), vis_offsets=np.array([0, m], dtype=np.int64),
        weight=np.ones(m, dtype=np.float32), flags=flags,
        beams=gaussian_pb(n_sky, pix, fwhm_deg * DEG)[None].astype(np.float32),
        interp=identity_interp(n_sky)[None].astype(np.float32),
        x_true=x, noise=noise, noise_rule=noise_rule,
        meta={"seed": seed, "freq_hz": freq_hz, "fwhm_deg": fwhm_deg},
        w=uvw[:, 2].astype(np.float32) if w_term else None,
    )


def config_c1(seed: int = 1001, lambda_r: float = 0.0) -> Problem:
    """64x64 sky, 10 arcsec pixels, 5 point sources U[0.1,1] Jy, 1 deg PB, 36-antenna
    6 km array at 1.4 GHz over 6 h, first 20,000 visibilities, sigma = 0.01 Jy."""
    return single_pointing("c1-points-64", seed, 64, 10.0, 32, 20_000, "points", lambda_r,
                           ("abs", 0.01))


def config_c2(seed: int = 2001, n_time: int = 1000, n_sky: int = 512) -> Problem:
    """512x512 sky at 7 arcsec of a k^-3 log-normal field (0-50 K), 630 baselines x 1000
    samples = 630,000 visibilities, noise 1% of peak, lambda_r = 1e-2."""
    return single_pointing("c2-diffuse-512", seed, n_sky, 7.0, n_time, None, "diffuse", 1e-2,
                           ("frac_peak", 0.01))


def mosaic(name: str, seed: int, n_sky: int, pixel_arcsec: float, n_rows: int, n_cols: int,
           pitch_px: float, fwhm_px: float, n_sub: int, time_range, flag_max: float,
           n_chan: int = 1, lambda_r: float = 1e-2, lambda_s: float = 1.0,
           sd_n: int = 64, sd_fwhm_arcmin: float = 16.0, freq_hz: float = 1.4e9,
           n_keep: Optional[int] = None, max_vis_per_block: Optional[int] = None,
           w_term: bool = False) -> Problem:
    """Hexagonal mosaic of Gaussian-beam pointings over one sky (Sect. 4.4 geometry):
    each pointing has its own track length T_k ~ U{time_range} and flag rate
    f_k ~ U[0, flag_max] (Bernoulli per visibility), giving uneven counts.  w_term: the
    problem carries the w coordinate of every sample (the full model of Eq. vis)."""
    st = _streams(seed, _STREAMS)
    pix = pixel_arcsec * ARCSEC
    enu = antenna_layout(st["layout"], 36, 3000.0)
    bl = baselines(enu)
    centres = hex_centres(n_rows, n_cols, pitch_px, n_sky)
    P = centres.shape[0]
    if n_chan == 1:
        x = lognormal_field(grf_k3(st["field"], n_sky))[None]
    else:
        x = ar1_cube(st["field"], n_chan, n_sky)
    beams, grids, uvs, ws, flags, offs = [], [], [], [], [], [0]
    pb = gaussian_pb(n_sub, pix, fwhm_px * pix)
    for k in range(P):
        g, (rak, deck) = sin_interp(n_sky, n_sub, pix, centres[k])
        grids.append(g)
        beams.append(pb)
        n_t = int(st["tracks"].integers(time_range[0], time_range[1] + 1))
        uvwk = uvw_tracks(bl, n_t, deck, freq_hz)
        if n_keep is not None:
            uvwk = uvwk[:n_keep]
        if max_vis_per_block is not None:
            uvwk = uvwk[:max_vis_per_block]
        uvk = uvwk[:, :2]
        fr = st["flags"].uniform(0.0, flag_max)
        for c in range(n_chan):
            uvs.append(uvk)
            ws.append(uvwk[:, 2])
            flags.append((st["flags"].uniform(size=uvk.shape[0]) < fr).astype(np.uint8))
            offs.append(offs[-1] + uvk.shape[0])
    uv = np.concatenate(uvs).astype(np.float32)
    m = uv.shape[0]
    noise = st["noise"].standard_normal(m) + 1j * st["noise"].standard_normal(m)
    sd_stride = n_sky // sd_n if sd_n else 0
    return Problem(
        name=name, n_chan=n_chan, n_sky=n_sky, pixel_rad=pix, n_point=P, n_sub=n_sub,
        flux_scale=np.full(n_chan, rj_flux_scale(freq_hz, pix)), lambda_r=lambda_r,
        lambda_s=lambda_s, uv=uv, vis_offsets=np.array(offs, dtype=np.int64),
        weight=np.ones(m, dtype=np.float32), flags=np.concatenate(flags),
        beams=np.stack(beams).astype(np.float32), interp=np.stack(grids).astype(np.float32),
        x_true=x, noise=noise, noise_rule=("frac_peak", 0.01),
        sd_n=sd_n, sd_stride=sd_stride, sd_offset=sd_stride // 2,
        sd_fwhm_rad=sd_fwhm_arcmin * ARCMIN,
        meta={"seed": seed, "freq_hz": freq_hz, "centres": centres, "fwhm_rad": fwhm_px * pix},
        w=np.concatenate(ws).astype(np.float32) if w_term else None,
    )


def config_c3(seed: int = 3001, time_range=(1400, 2000), n_keep=None, w_term: bool = False) -> Problem:
    """36 pointings (6x6 hex, 1 deg pitch = 120 px at 30 arcsec) over a 1024^2 sky, 1 deg
    PB, 384^2 sub-images, T_k ~ U{1400..2000} samples x 630 baselines, 0-30% flags,
    64x64 single-dish map under a 16 arcmin beam, lambda_r = 1e-2, lambda_s = 1."""
    return mosaic("c3-mosaic-36x1024", seed, 1024, 30.0, 6, 6, 120.0, 120.0, 384, time_range,
                  0.3, n_keep=n_keep, w_term=w_term)


def config_c3_mini(seed: int = 3101, w_term: bool = False) -> Problem:
    """Reduced mosaic with the C3 structure (hex footprint, SIN grids, uneven flagged
    counts, SD map) at a size the oracle evaluates in seconds: 2x2 pointings, 128^2 sky,
    64^2 sub-images, 30-60 samples x 630 baselines."""
    return mosaic("c3-mini", seed, 128, 30.0, 2, 2, 30.0, 30.0, 64, (30, 60), 0.3,
                  sd_n=16, sd_fwhm_arcmin=4.0, w_term=w_term)


def config_w_single(seed: int = 6001, n_sky: int = 64, pixel_arcsec: float = 60.0, n_time: int = 8) -> Problem:
    """Single pointing with the w coordinate of every sample (the full model of Eq. vis) on a
    wide field: 64^2 sky at 60 arcsec (a 64 arcmin sub-image, 0.75 deg to the corners, where
    the phase the coplanar model drops reaches several radians on the long baselines),
    630 baselines x 8 samples, k^-3 log-normal sky, noise 1% of peak, lambda_r = 1e-2."""
    return single_pointing("w-single-64", seed, n_sky, pixel_arcsec, n_time, None, "diffuse", 1e-2,
                           ("frac_peak", 0.01), w_term=True)


def config_c5_geometry(seed: int = 5001) -> Problem:
    """Warm-start geometry: 256^2 sky at 30 arcsec, 3x3 hex of 20 arcmin beams (pitch
    40 px), 128^2 sub-images, 200,000 visibilities per pointing, lambda_s = 0."""
    return mosaic("c5-warmstart-256", seed, 256, 30.0, 3, 3, 40.0, 40.0, 128, (318, 318), 0.0,
                  lambda_s=0.0, sd_n=0, max_vis_per_block=200_000)


# ----------------------------------------------------------------------------- cubes

@dataclass
class CubeProblem:
    """Spectral cube whose channels share each pointing's uv track and weights (the same
    baselines observed at every frequency): channel c of pointing k sees
    uv[pt_offsets[k]:pt_offsets[k+1]] * uv_scale[c].  Visibilities and flags are stored per
    (pointing, channel) block, block index k * n_chan + c, every channel of pointing k
    holding M_k samples."""

    name: str
    n_chan: int
    n_sky: int
    pixel_rad: float
    n_point: int
    n_sub: int
    flux_scale: np.ndarray  # [C] float64
    lambda_r: float
    lambda_s: float
    uv: np.ndarray  # [sum M_k, 2] float32, wavelengths at the reference frequency
    pt_offsets: np.ndarray  # [P + 1] int64
    uv_scale: np.ndarray  # [C] float64, nu_c / nu_ref
    weight: np.ndarray  # [sum M_k] float32
    vis_offsets: np.ndarray  # [P*C + 1] int64
    flags: np.ndarray  # [M] uint8
    beams: np.ndarray
    interp: np.ndarray
    x_true: Optional[np.ndarray]  # [C][N][N] float32, or None
    vis: np.ndarray  # [M] complex64: unit-variance complex noise
    sd_n: int = 0
    sd_stride: int = 0
    sd_offset: int = 0
    sd_fwhm_rad: float = 0.0
    sd_sigma: float = 0.0
    sd_map: Optional[np.ndarray] = None
    sd_noise_frac: float = 0.01
    lambda_nu: float = 0.0  # spectral smoothness weight (couples adjacent channels)
    meta: dict = field(default_factory=dict)
    w: Optional[np.ndarray] = None  # [sum M_k] float32 at the reference frequency, or None

    @property
    def n_vis(self) -> int:
        return int(self.vis_offsets[-1])

    @property
    def n_items(self) -> int:
        return self.n_point * self.n_chan

    def block(self, k: int, c: int) -> slice:
        i = k * self.n_chan + c
        return slice(int(self.vis_offsets[i]), int(self.vis_offsets[i + 1]))

    def w_of(self, k: int, c: int) -> Optional[np.ndarray]:
        """FP64 w of block (k, c) at the channel's frequency, or None (coplanar model)."""
        if self.w is None:
            return None
        s = slice(int(self.pt_offsets[k]), int(self.pt_offsets[k + 1]))
        return self.w[s].astype(np.float64) * self.uv_scale[c]

    def uv_of(self, k: int, c: int) -> np.ndarray:
        """FP64 uv of block (k, c), wavelengths at the channel's frequency."""
        s = slice(int(self.pt_offsets[k]), int(self.pt_offsets[k + 1]))
        return self.uv[s].astype(np.float64) * self.uv_scale[c]

    def weight_of(self, k: int) -> np.ndarray:
        return self.weight[int(self.pt_offsets[k]):int(self.pt_offsets[k + 1])]

    def block_problem(self, k: int, c: int, x: Optional[np.ndarray] = None) -> Problem:
        """One (pointing, channel) block as a one-pointing, one-channel Problem with channel
        c's sky (x[c], or x_true[c]) and single-dish map."""
        s = self.block(k, c)
        xs = self.x_true if x is None else x
        xc = np.zeros((1, self.n_sky, self.n_sky)) if xs is None else np.asarray(xs[c:c + 1], dtype=np.float64)
        return Problem(
            name=f"{self.name}-k{k}-c{c}", n_chan=1, n_sky=self.n_sky, pixel_rad=self.pixel_rad, n_point=1,
            n_sub=self.n_sub, flux_scale=self.flux_scale[c:c + 1], lambda_r=self.lambda_r, lambda_s=self.lambda_s,
            uv=self.uv_of(k, c), vis_offsets=np.array([0, s.stop - s.start], dtype=np.int64),
            weight=self.weight_of(k), flags=self.flags[s], beams=self.beams[k:k + 1], interp=self.interp[k:k + 1],
            x_true=xc, noise=np.zeros(0), noise_rule=("abs", 1.0), sd_n=self.sd_n, sd_stride=self.sd_stride,
            sd_offset=self.sd_offset, sd_fwhm_rad=self.sd_fwhm_rad, sd_sigma=self.sd_sigma,
            sd_map=None if self.sd_map is None else self.sd_map[c:c + 1], sd_noise_frac=self.sd_noise_frac,
            vis=self.vis[s], meta=dict(self.meta), w=self.w_of(k, c))

    def expand(self) -> Problem:
        """The same data as a per-block Problem (FP64 uv per block); small cubes only."""
        uv = np.concatenate([self.uv_of(k, c) for k in range(self.n_point) for c in range(self.n_chan)])
        w = np.concatenate([self.weight_of(k) for k in range(self.n_point) for c in range(self.n_chan)])
        ww = None if self.w is None else np.concatenate(
            [self.w_of(k, c) for k in range(self.n_point) for c in range(self.n_chan)])
        x = self.x_true if self.x_true is not None else np.zeros((self.n_chan, self.n_sky, self.n_sky))
        return Problem(
            name=self.name, n_chan=self.n_chan, n_sky=self.n_sky, pixel_rad=self.pixel_rad,
            n_point=self.n_point, n_sub=self.n_sub, flux_scale=self.flux_scale, lambda_r=self.lambda_r,
            lambda_s=self.lambda_s, uv=uv, vis_offsets=self.vis_offsets, weight=w.astype(np.float32),
            flags=self.flags, beams=self.beams, interp=self.interp, x_true=np.asarray(x, dtype=np.float64),
            noise=np.zeros(0), noise_rule=("abs", 1.0), sd_n=self.sd_n, sd_stride=self.sd_stride,
            sd_offset=self.sd_offset, sd_fwhm_rad=self.sd_fwhm_rad, sd_sigma=self.sd_sigma,
            sd_map=self.sd_map, sd_noise_frac=self.sd_noise_frac, vis=self.vis, lambda_nu=self.lambda_nu,
            meta=dict(self.meta), w=ww)


def channel_freqs(n_chan: int, centre_hz: float, width_hz: float) -> np.ndarray:
    """Channel centre frequencies, symmetric about centre_hz."""
    return centre_hz + (np.arange(n_chan) - 0.5 * (n_chan - 1)) * width_hz


def cube(name: str, seed: int, n_sky: int, pixel_arcsec: float, n_rows: int, n_cols: int, pitch_px: float,
         fwhm_px: float, n_sub: int, n_time: int, n_chan: int, flag_max: float, centre_hz: float,
         width_hz: float, ref_hz: float = 1.4e9, lambda_r: float = 1e-2, lambda_s: float = 1.0,
         sd_n: int = 64, sd_fwhm_arcmin: float = 16.0, n_keep: Optional[int] = None, with_field: bool = True,
         threads: Optional[int] = None, w_term: bool = False) -> CubeProblem:
    """Hexagonal mosaic observed in n_chan channels: one uv track per pointing (n_time
    samples x 630 baselines at ref_hz, scaled by nu_c / ref_hz per channel), flag rate
    f_kc ~ U[0, flag_max] per (pointing, channel) with Bernoulli flags, channel-correlated
    log-normal cube (AR(1), rho = 0.9), Rayleigh-Jeans flux scale per channel.  The
    visibilities are unit-variance complex noise; flags and noise of block b are drawn
    from SeedSequence([seed, b]) so the blocks can be filled by parallel threads.  w_term:
    each track also carries its w coordinate (the full model of Eq. vis)."""
    from concurrent.futures import ThreadPoolExecutor

    st = _streams(seed, _STREAMS)
    pix = pixel_arcsec * ARCSEC
    enu = antenna_layout(st["layout"], 36, 3000.0)
    bl = baselines(enu)
    centres = hex_centres(n_rows, n_cols, pitch_px, n_sky)
    P = centres.shape[0]
    x = ar1_cube(st["field"], n_chan, n_sky).astype(np.float32) if with_field else None
    pb = gaussian_pb(n_sub, pix, fwhm_px * pix)
    grids, uvs, ws, pt = [], [], [], [0]
    for k in range(P):
        g, (rak, deck) = sin_interp(n_sky, n_sub, pix, centres[k])
        grids.append(g)
        uvwk = uvw_tracks(bl, n_time, deck, ref_hz)
        if n_keep is not None:
            uvwk = uvwk[:n_keep]
        uvs.append(uvwk[:, :2])
        ws.append(uvwk[:, 2])
        pt.append(pt[-1] + uvwk.shape[0])
    freqs = channel_freqs(n_chan, centre_hz, width_hz)
    rates = st["flags"].uniform(0.0, flag_max, size=(P, n_chan))
    mk = np.diff(np.array(pt))
    offs = np.concatenate([[0], np.cumsum(np.repeat(mk, n_chan))]).astype(np.int64)
    m = int(offs[-1])
    flags = np.empty(m, dtype=np.uint8)
    vis = np.empty(m, dtype=np.complex64)
    vf = vis.view(np.float32)

    def fill(b: int):
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, b])))
        k, c = divmod(b, n_chan)
        a, e = int(offs[b]), int(offs[b + 1])
        flags[a:e] = rng.random(e - a, dtype=np.float32) < rates[k, c]
        rng.standard_normal(2 * (e - a), dtype=np.float32, out=vf[2 * a:2 * e])

    with ThreadPoolExecutor(max_workers=threads or min(16, max(1, P * n_chan))) as ex:
        list(ex.map(fill, range(P * n_chan)))
    sd_stride = n_sky // sd_n if sd_n else 0
    return CubeProblem(
        name=name, n_chan=n_chan, n_sky=n_sky, pixel_rad=pix, n_point=P, n_sub=n_sub,
        flux_scale=np.array([rj_flux_scale(f, pix) for f in freqs]), lambda_r=lambda_r, lambda_s=lambda_s,
        uv=np.concatenate(uvs).astype(np.float32), pt_offsets=np.array(pt, dtype=np.int64),
        uv_scale=freqs / ref_hz, weight=np.ones(pt[-1], dtype=np.float32), vis_offsets=offs, flags=flags,
        beams=np.repeat(pb[None], P, axis=0).astype(np.float32), interp=np.stack(grids).astype(np.float32),
        x_true=x, vis=vis, sd_n=sd_n, sd_stride=sd_stride, sd_offset=sd_stride // 2,
        sd_fwhm_rad=sd_fwhm_arcmin * ARCMIN,
        meta={"seed": seed, "freqs": freqs, "ref_hz": ref_hz, "centres": centres, "flag_rates": rates},
        w=np.concatenate(ws).astype(np.float32) if w_term else None,
    )


def config_c4(seed: int = 4001, n_chan: int = 128, n_time: int = 1800, with_field: bool = True,
              threads: Optional[int] = None) -> CubeProblem:
    """Spectral cube on the 36-pointing mosaic geometry: 128 channels of 2.315 kHz around
    1402 MHz, 630 baselines x 1800 samples per pointing (1,134,000 per (pointing,
    channel), about 5.2e9 in all), 0-5% flags per (pointing, channel), 64x64 single-dish
    map per channel, lambda_r = 1e-2, lambda_s = 1."""
    return cube("c4-cube-128x36x1024", seed, 1024, 30.0, 6, 6, 120.0, 120.0, 384, n_time, n_chan, 0.05,
                1402e6, 2.315e3, with_field=with_field, threads=threads)


def config_c4_mini(seed: int = 4101, w_term: bool = False) -> CubeProblem:
    """The cube structure at a size the oracle evaluates in seconds: 2x2 pointings on a
    128^2 sky, 64^2 sub-images, 4 channels 25 MHz apart (uv scales 0.97-1.03, so a wrong
    channel scale shows), 40 samples x 630 baselines per pointing, 0-30% flags."""
    return cube("c4-mini", seed, 128, 30.0, 2, 2, 30.0, 30.0, 64, 40, 4, 0.3, 1.4e9, 25e6,
                sd_n=16, sd_fwhm_arcmin=4.0, w_term=w_term)


CONFIGS = {
    "c1": config_c1,
    "c2": config_c2,
    "c3": config_c3,
    "c3-mini": config_c3_mini,
    "c5": config_c5_geometry,
    "c4": config_c4,
    "c4-mini": config_c4_mini,
}
