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
