"""FP64 oracle of the data processor: SIN interpolation grids, their inverse (deprojection)
grids and primary-beam resampling (Sect. 3.3; Eq. sin_projection, Eq. sin_deprojection).

TEST INFRASTRUCTURE: only tests/ may import this module.  It shares no code with the HIP path.

The orthographic (SIN) projection about a centre (ra0, dec0) is written here with direction
vectors: a direction e = (cos dec cos ra, cos dec sin ra, sin dec) has direction cosines
l = e . east, m = e . north, n = e . centre in the basis of the tangent point (Calabretta &
Greisen 2002, the SIN projection of the paper's reference); the inverse is
e = l east + m north + sqrt(1 - l^2 - m^2) centre.  Frames: pixel (row, col) of an image
with pixel size delta centred on (ra0, dec0) has l = (col - c0) delta, m = (row - r0) delta
with the reference pixel (r0, c0) = (n/2, n/2); l runs along columns, m along rows, no sign
flip (the library's reading of the pixel <-> (l, m) mapping).
"""
from __future__ import annotations

import numpy as np


def basis(ra0: float, dec0: float):
    """East, north and centre unit vectors of the tangent point (ra0, dec0)."""
    east = np.array([-np.sin(ra0), np.cos(ra0), 0.0])
    north = np.array([-np.sin(dec0) * np.cos(ra0), -np.sin(dec0) * np.sin(ra0), np.cos(dec0)])
    centre = np.array([np.cos(dec0) * np.cos(ra0), np.cos(dec0) * np.sin(ra0), np.sin(dec0)])
    return east, north, centre


def direction(ra, dec):
    """Unit vectors of (ra, dec) arrays, shape [..., 3]."""
    ra, dec = np.asarray(ra, dtype=np.float64), np.asarray(dec, dtype=np.float64)
    return np.stack([np.cos(dec) * np.cos(ra), np.cos(dec) * np.sin(ra), np.sin(dec)], axis=-1)


def radec(e):
    """(ra, dec) of unit vectors [..., 3]."""
    e = np.asarray(e, dtype=np.float64)
    return np.arctan2(e[..., 1], e[..., 0]), np.arcsin(np.clip(e[..., 2], -1.0, 1.0))


def project(e, ra0, dec0):
    """(l, m, n) of directions e about (ra0, dec0)."""
    east, north, centre = basis(ra0, dec0)
    return e @ east, e @ north, e @ centre


def unproject(l, m, ra0, dec0):
    """Directions of (l, m) on the near hemisphere of (ra0, dec0)."""
    east, north, centre = basis(ra0, dec0)
    l, m = np.asarray(l, dtype=np.float64), np.asarray(m, dtype=np.float64)
    n = np.sqrt(np.maximum(0.0, 1.0 - l * l - m * m))
    return l[..., None] * east + m[..., None] * north + n[..., None] * centre


def pixel_lm(n_pix: int, delta: float):
    """(L, M) of every pixel of an n x n image: L[a, b] = (b - n/2) delta, M[a, b] = (a - n/2) delta."""
    t = (np.arange(n_pix) - n_pix // 2) * delta
    return np.meshgrid(t, t)


def sin_grid(n_sky: int, sky_delta: float, ra0: float, dec0: float, n_sub: int, sub_delta: float,
             ra_k: float, dec_k: float) -> np.ndarray:
    """Interpolation grid of pointing k: [n_sub][n_sub][2] (row, col) of the sky-image
    position seen by every sub-pixel of pointing k's SIN image."""
    L, M = pixel_lm(n_sub, sub_delta)
    l, m, _ = project(unproject(L, M, ra_k, dec_k), ra0, dec0)
    return np.stack([m / sky_delta + n_sky // 2, l / sky_delta + n_sky // 2], axis=-1)


def deprojection_grid(n_sky: int, sky_delta: float, ra0: float, dec0: float, n_sub: int, sub_delta: float,
                      ra_k: float, dec_k: float):
    """Inverse of sin_grid: [n_sky][n_sky][2] (row, col) in pointing k's sub-image of every
    sky pixel, and a mask of the pixels on pointing k's near hemisphere (n > 0)."""
    L, M = pixel_lm(n_sky, sky_delta)
    l, m, n = project(unproject(L, M, ra0, dec0), ra_k, dec_k)
    g = np.stack([m / sub_delta + n_sub // 2, l / sub_delta + n_sub // 2], axis=-1)
    return g, n > 0.0


def bilinear(img: np.ndarray, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """Bilinear sample of img at (rows, cols); pixel (i, j) sits at (i, j); pixels outside
    the image contribute 0 (the reprojection convention of the forward model)."""
    img = np.asarray(img, dtype=np.float64)
    h, w = img.shape
    i0, j0 = np.floor(rows).astype(np.int64), np.floor(cols).astype(np.int64)
    fy, fx = rows - i0, cols - j0
    out = np.zeros(np.shape(rows))
    for di, dj, wt in ((0, 0, (1 - fy) * (1 - fx)), (0, 1, (1 - fy) * fx), (1, 0, fy * (1 - fx)), (1, 1, fy * fx)):
        ii, jj = i0 + di, j0 + dj
        ok = (ii >= 0) & (ii < h) & (jj >= 0) & (jj < w)
        out += np.where(ok, wt * img[np.clip(ii, 0, h - 1), np.clip(jj, 0, w - 1)], 0.0)
    return out


def resample_beam(beam: np.ndarray, beam_delta: float, n_sub: int, sub_delta: float) -> np.ndarray:
    """A beam image of pixel size beam_delta (peak at its reference pixel (nb/2, nb/2), the
    pointing centre) resampled onto the n_sub x n_sub sub-image grid of pixel size sub_delta:
    sub-pixel (a, b) at (l, m) reads the beam at (m / beam_delta + nb/2, l / beam_delta + nb/2)
    (bilinear, 0 outside the beam image)."""
    nb = beam.shape[0]
    L, M = pixel_lm(n_sub, sub_delta)
    return bilinear(beam, M / beam_delta + nb // 2, L / beam_delta + nb // 2)


def linear_mosaic(sub_images: np.ndarray, beams: np.ndarray, deproj: np.ndarray, pb_min: float = 0.0):
    """Eq. linear and Eq. pb_eff (Sect. 4.4.1): every pointing's image I'_k (sub_images
    [P][C][n][n]) and beam A_k ([P][n][n]) are sampled at the sky pixels' positions in its
    sub-image (deproj [P][N][N][2], Eq. sin_deprojection; bilinear, 0 outside), and
    I = sum_k A_k^2 I'_k / sum_k A_k^2 where sqrt(sum_k A_k^2) >= pb_min (0 elsewhere);
    A_eff = sqrt(sum_k A_k^2).  Returns (image [C][N][N], A_eff [N][N])."""
    P, C = sub_images.shape[:2]
    N = deproj.shape[1]
    num = np.zeros((C, N, N))
    den = np.zeros((N, N))
    for k in range(P):
        rows, cols = deproj[k][..., 0].astype(np.float64), deproj[k][..., 1].astype(np.float64)
        A = bilinear(beams[k], rows, cols)
        den += A * A
        for c in range(C):
            num[c] += A * A * bilinear(sub_images[k, c], rows, cols)
    keep = (den > 0) & (den >= pb_min * pb_min)
    image = np.where(keep[None], num / np.where(keep, den, 1.0)[None], 0.0)
    return image, np.sqrt(den)


def feather_transfer(n: int, delta: float, theta: float) -> np.ndarray:
    """B(k) = exp(-2 pi^2 sigma^2 |k|^2), sigma = theta / (2 sqrt(2 ln 2)) (App. B), on the
    n x n FFT frequency grid of pixel size delta (cycles per radian)."""
    sigma = theta / (2.0 * np.sqrt(2.0 * np.log(2.0)))
    f = np.fft.fftfreq(n, d=delta)
    k2 = f[:, None] ** 2 + f[None, :] ** 2
    return np.exp(-2.0 * np.pi ** 2 * sigma ** 2 * k2)


def feather(interf: np.ndarray, single_dish: np.ndarray, delta: float, theta: float) -> np.ndarray:
    """App. B: I_comb = F^-1[B F[I_SD] + (1 - B) F[I_int]] per channel ([C][n][n] maps)."""
    interf = np.asarray(interf, dtype=np.float64)
    single_dish = np.asarray(single_dish, dtype=np.float64)
    B = feather_transfer(interf.shape[-1], delta, theta)
    out = np.empty_like(interf)
    for c in range(interf.shape[0]):
        comb = B * np.fft.fft2(single_dish[c]) + (1.0 - B) * np.fft.fft2(interf[c])
        out[c] = np.fft.ifft2(comb).real
    return out
