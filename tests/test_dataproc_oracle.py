"""Pins of the data-processor oracle (CPU): the SIN projection against its trigonometric
closed form, identity and round-trip properties, and beam resampling special cases."""
import numpy as np
import pytest

from oracle import dataproc as D

ARCSEC = np.pi / (180 * 3600)
DEG = np.pi / 180


def _trig_project(ra, dec, ra0, dec0):
    # the textbook SIN formulas (Calabretta & Greisen 2002, orthographic projection)
    l = np.cos(dec) * np.sin(ra - ra0)
    m = np.sin(dec) * np.cos(dec0) - np.cos(dec) * np.sin(dec0) * np.cos(ra - ra0)
    return l, m


def test_projection_matches_the_trigonometric_form():
    rng = np.random.default_rng(1)
    ra0, dec0 = 1.37, -1.2
    ra = ra0 + rng.uniform(-0.2, 0.2, 500)
    dec = dec0 + rng.uniform(-0.2, 0.2, 500)
    l, m, n = D.project(D.direction(ra, dec), ra0, dec0)
    lt, mt = _trig_project(ra, dec, ra0, dec0)
    np.testing.assert_allclose(l, lt, atol=1e-15)
    np.testing.assert_allclose(m, mt, atol=1e-15)
    np.testing.assert_allclose(l * l + m * m + n * n, 1.0, atol=1e-15)
    # the tangent point projects to the origin; north of it has l = 0, m > 0
    l0, m0, n0 = D.project(D.direction(ra0, dec0), ra0, dec0)
    assert abs(l0) < 1e-16 and abs(m0) < 1e-16 and n0 == pytest.approx(1.0)
    ln, mn, _ = D.project(D.direction(ra0, dec0 + 0.01), ra0, dec0)
    assert abs(ln) < 1e-16 and mn == pytest.approx(np.sin(0.01), rel=1e-14)


def test_unproject_inverts_project():
    rng = np.random.default_rng(2)
    ra0, dec0 = 5.6, -0.3
    l, m = rng.uniform(-0.05, 0.05, (2, 300))
    l2, m2, _ = D.project(D.unproject(l, m, ra0, dec0), ra0, dec0)
    np.testing.assert_allclose(l2, l, atol=1e-16)
    np.testing.assert_allclose(m2, m, atol=1e-16)
    ra, dec = D.radec(D.unproject(l, m, ra0, dec0))
    l3, m3 = _trig_project(ra, dec, ra0, dec0)
    np.testing.assert_allclose(l3, l, atol=1e-15)


def test_grid_of_the_central_pointing_is_a_translation():
    """A pointing at the sky frame's centre with the same pixel size samples the sky at
    (a - n/2 + N/2, b - n/2 + N/2): the crop of the coplanar case."""
    ra0, dec0 = 1.38, -1.205
    g = D.sin_grid(256, 30 * ARCSEC, ra0, dec0, 64, 30 * ARCSEC, ra0, dec0)
    a = np.arange(64)
    np.testing.assert_allclose(g[..., 0], (a - 32 + 128)[:, None] + 0 * a[None, :], atol=1e-9)
    np.testing.assert_allclose(g[..., 1], (a - 32 + 128)[None, :] + 0 * a[:, None], atol=1e-9)


def test_grid_and_deprojection_are_inverse():
    ra0, dec0 = 1.38, -1.205
    dsky, dsub = 30 * ARCSEC, 30 * ARCSEC
    rak, deck = ra0 + 0.8 * DEG / np.cos(dec0), dec0 - 0.5 * DEG
    g = D.sin_grid(1024, dsky, ra0, dec0, 384, dsub, rak, deck)
    dg, near = D.deprojection_grid(1024, dsky, ra0, dec0, 384, dsub, rak, deck)
    assert near.all()
    # follow sub-pixel (a, b) to the sky and back (bilinear of the inverse grid is exact to
    # its curvature: compare at the integer sky pixel nearest to a few sub-pixels instead)
    for a, b in ((0, 0), (100, 250), (383, 17), (192, 192)):
        r, c = g[a, b]
        i, j = int(np.floor(r)), int(np.floor(c))
        back = D.bilinear(dg[..., 0], np.array(r), np.array(c)), D.bilinear(dg[..., 1], np.array(r), np.array(c))
        assert abs(back[0] - a) < 1e-4 and abs(back[1] - b) < 1e-4
    # the pointing centre maps to the sub-image's reference pixel
    l, m, _ = D.project(D.direction(rak, deck), ra0, dec0)
    rc, cc = m / dsky + 512, l / dsky + 512
    assert D.bilinear(dg[..., 0], np.array(rc), np.array(cc)) == pytest.approx(192, abs=1e-6)
    assert D.bilinear(dg[..., 1], np.array(rc), np.array(cc)) == pytest.approx(192, abs=1e-6)


def test_beam_resampling_special_cases():
    rng = np.random.default_rng(3)
    beam = rng.uniform(0.0, 1.0, (64, 64))
    # same pixel size and size: a copy
    np.testing.assert_allclose(D.resample_beam(beam, 30 * ARCSEC, 64, 30 * ARCSEC), beam, rtol=0, atol=1e-14)
    # bilinear is exact on a linear function: a plane beam resampled at any scale stays the plane
    i, j = np.meshgrid(np.arange(128.0), np.arange(128.0), indexing="ij")
    plane = 0.3 + 0.01 * i - 0.002 * j
    out = D.resample_beam(plane, 20 * ARCSEC, 96, 30 * ARCSEC)
    a, b = np.meshgrid(np.arange(96.0), np.arange(96.0), indexing="ij")
    rows, cols = (a - 48) * 1.5 + 64, (b - 48) * 1.5 + 64
    want = np.where((rows <= 127) & (cols <= 127) & (rows >= 0) & (cols >= 0), 0.3 + 0.01 * rows - 0.002 * cols, np.nan)
    ok = ~np.isnan(want) & (rows < 127) & (cols < 127)
    np.testing.assert_allclose(out[ok], want[ok], atol=1e-14)
    # outside the beam image: 0
    assert D.resample_beam(beam, 1 * ARCSEC, 64, 30 * ARCSEC)[0, 0] == 0.0


def test_feather_special_cases():
    """B(0) = 1 and B + (1 - B) = 1: equal maps come back unchanged and the total flux is the
    single dish's; one Fourier mode of the interferometric map alone is scaled by 1 - B(k),
    with B(k) = exp(-2 pi^2 sigma^2 k^2), sigma = theta / (2 sqrt(2 ln 2)); theta = 0 keeps
    the single-dish map."""
    rng = np.random.default_rng(4)
    n, delta, theta = 64, 30 * ARCSEC, 20 * 60 * ARCSEC
    a = rng.standard_normal((2, n, n))
    np.testing.assert_allclose(D.feather(a, a, delta, theta), a, atol=1e-12)
    sd = rng.standard_normal((1, n, n)) + 3.0
    out = D.feather(a[:1], sd, delta, theta)
    assert out.mean() == pytest.approx(sd.mean(), rel=1e-12)
    p, q = 5, 3
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    mode = np.cos(2 * np.pi * (q * i + p * j) / n)[None]
    sigma = theta / (2 * np.sqrt(2 * np.log(2)))
    k2 = (p * p + q * q) / (n * delta) ** 2
    want = (1 - np.exp(-2 * np.pi ** 2 * sigma ** 2 * k2)) * mode
    np.testing.assert_allclose(D.feather(mode, np.zeros_like(mode), delta, theta), want, atol=1e-12)
    np.testing.assert_allclose(D.feather(a[:1], sd, delta, 0.0), sd, atol=1e-12)


def test_linear_mosaic_special_cases():
    """One pointing under a constant beam returns its (deprojected) image, a plane being
    sampled exactly; pointings that all see the same constant give that constant wherever
    covered; A_eff is sqrt(sum A_k^2); pixels below pb_min are 0."""
    ra0, dec0 = 1.38, -1.205
    d = 30 * ARCSEC
    N, n = 96, 48
    dg, _ = D.deprojection_grid(N, d, ra0, dec0, n, d, ra0, dec0)
    a, b = np.meshgrid(np.arange(n, dtype=float), np.arange(n, dtype=float), indexing="ij")
    plane = 1.0 + 0.02 * a - 0.01 * b
    img, peff = D.linear_mosaic(plane[None, None], np.full((1, n, n), 0.5), dg[None])
    inner = (dg[..., 0] >= 0) & (dg[..., 0] <= n - 1) & (dg[..., 1] >= 0) & (dg[..., 1] <= n - 1)
    want = 1.0 + 0.02 * dg[..., 0] - 0.01 * dg[..., 1]
    np.testing.assert_allclose(img[0][inner], want[inner], atol=1e-12)
    np.testing.assert_allclose(peff[inner], 0.5, atol=1e-14)
    rak = ra0 + 4 * d / np.cos(dec0)
    dg2, _ = D.deprojection_grid(N, d, ra0, dec0, n, d, rak, dec0)
    beams = np.stack([np.full((n, n), 0.5), np.full((n, n), 0.8)])
    img, peff = D.linear_mosaic(np.full((2, 1, n, n), 3.0), beams, np.stack([dg, dg2]))
    # pixels whose bilinear taps lie wholly inside or wholly outside each sub-image (at an edge
    # the zero padding weighs beam and image alike, so their ratio is not the constant)
    clean = np.ones((N, N), dtype=bool)
    for g in (dg, dg2):
        inside = (g[..., 0] >= 0) & (g[..., 0] <= n - 1) & (g[..., 1] >= 0) & (g[..., 1] <= n - 1)
        outside = (g[..., 0] <= -1) | (g[..., 0] >= n) | (g[..., 1] <= -1) | (g[..., 1] >= n)
        clean &= inside | outside
    both = clean & (peff > 0)
    assert both.sum() > 1000
    np.testing.assert_allclose(img[0][both], 3.0, atol=1e-12)
    np.testing.assert_allclose(peff[both & (np.abs(dg2[..., 0] - 24) < 20) & (np.abs(dg[..., 0] - 24) < 20)
                                    & (np.abs(dg2[..., 1] - 24) < 20) & (np.abs(dg[..., 1] - 24) < 20)],
                               np.sqrt(0.25 + 0.64), atol=1e-12)
    img, _ = D.linear_mosaic(np.full((2, 1, n, n), 3.0), beams, np.stack([dg, dg2]), pb_min=0.9)
    assert np.all(img[0][peff < 0.9] == 0.0) and np.all(np.abs(img[0][both & (peff >= 0.9)] - 3.0) < 1e-12)
