"""Pins of the FP64 oracle against what the paper and the mathematics fix (CPU only).

Each test checks the oracle against something other than itself: printed values
(tests/golden), closed forms, textbook/library special cases, invariants, brute force
on tiny inputs and finite differences.  A plausible slip (dropped factor, wrong sign,
swapped axis, transposed operand) fails at least one of them.
"""
import cmath
import math
import os

import numpy as np
import pytest
import scipy.ndimage
import scipy.signal

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([float(t) for t in line.split()])
    return np.array(rows)


def _rand_uv(rng, m, delta, span=3.0):
    """uv with |u delta| up to `span` cycles per pixel: well beyond Nyquist (wraps)."""
    return rng.uniform(-span, span, size=(m, 2)) / delta


# ----------------------------------------------------------------------------- O3 / O5

def test_dft_hand_cases(oracle_mod):
    for n, a, b, flux, ud, vd, re, im in _golden("dft_hand_cases.txt"):
        n, a, b = int(n), int(a), int(b)
        f = np.zeros((n, n))
        f[a, b] = flux
        delta = 1e-4
        v = oracle_mod.dft_forward(f, np.array([[ud / delta, vd / delta]]), delta)[0]
        assert abs(v - complex(re, im)) < 1e-12, (n, a, b, v)


def test_point_source_at_phase_centre_is_flat(oracle_mod):
    """Closed form: a source of flux S at the phase centre under a unit-peak beam gives
    V_j = s S for every baseline, including uv beyond the pixel grid's Nyquist."""
    rng = np.random.default_rng(1)
    n, delta = 32, 10 * synth.ARCSEC
    pb = synth.gaussian_pb(n, delta, synth.DEG)
    assert pb[n // 2, n // 2] == 1.0
    f = np.zeros((n, n))
    f[n // 2, n // 2] = 0.7
    f = 2.5 * pb * f
    v = oracle_mod.dft_forward(f, _rand_uv(rng, 500, delta), delta)
    np.testing.assert_allclose(v, 2.5 * 0.7, rtol=0, atol=1e-13)


def test_point_source_off_centre_closed_form(oracle_mod):
    """A source at pixel (a, b) gives s S A[a,b] exp(-2 pi i (u l_b + v m_a)) with the
    phase taken directly (no fractional-part reduction) on in-band uv."""
    rng = np.random.default_rng(2)
    n, delta = 16, 7 * synth.ARCSEC
    a, b = 3, 11
    f = np.zeros((n, n))
    f[a, b] = 1.3
    uv = rng.uniform(-0.5, 0.5, size=(64, 2)) / delta
    v = oracle_mod.dft_forward(f, uv, delta)
    l, m = (b - n // 2) * delta, (a - n // 2) * delta
    want = 1.3 * np.exp(-2j * np.pi * (uv[:, 0] * l + uv[:, 1] * m))
    np.testing.assert_allclose(v, want, rtol=0, atol=1e-12)


def test_integer_frequencies_reduce_to_fft2(oracle_mod):
    """Textbook special case: u = p/(n delta), v = q/(n delta) on integer (p, q) makes the
    direct sum a DFT: V(p, q) = (-1)^(p+q) * fft2(f)[q, p] (numpy, FP64).  Pins the sign
    and which image axis pairs with u (columns) and v (rows)."""
    rng = np.random.default_rng(3)
    n, delta = 8, 1e-4
    f = rng.standard_normal((n, n))
    q, p = np.meshgrid(np.arange(-n, n), np.arange(-n, n), indexing="ij")
    uv = np.stack([p.ravel() / (n * delta), q.ravel() / (n * delta)], axis=1)
    v = oracle_mod.dft_forward(f, uv, delta).reshape(q.shape)
    F = np.fft.fft2(f)
    want = ((-1.0) ** (p + q)) * F[q % n, p % n]
    np.testing.assert_allclose(v, want, rtol=0, atol=1e-11)


def test_brute_force_tiny(oracle_mod):
    """4x4 sub-image, 3 visibilities: pure-Python complex exponentials of the full phase
    (no fractional-part reduction, no separable factors) vs the C oracle."""
    rng = np.random.default_rng(4)
    n, delta = 4, 12 * synth.ARCSEC
    f = rng.standard_normal((n, n))
    uv = np.array([[1234.5, -987.25], [-40000.0, 51234.0], [0.0, 77.0]])
    coef = np.array([0.3 - 1.1j, 2.0 + 0.5j, -0.7 + 0.25j])
    vb = []
    for u, v in uv:
        s = 0j
        for a in range(n):
            for b in range(n):
                l, m = (b - n / 2) * delta, (a - n / 2) * delta
                s += f[a, b] * cmath.exp(-2j * math.pi * (u * l + v * m))
        vb.append(s)
    gb = np.zeros((n, n))
    for a in range(n):
        for b in range(n):
            l, m = (b - n / 2) * delta, (a - n / 2) * delta
            gb[a, b] = sum((c * cmath.exp(2j * math.pi * (u * l + v * m))).real
                           for c, (u, v) in zip(coef, uv))
    np.testing.assert_allclose(oracle_mod.dft_forward(f, uv, delta), vb, rtol=0, atol=1e-12)
    np.testing.assert_allclose(oracle_mod.dft_adjoint(coef, uv, delta, n), gb, rtol=0, atol=1e-12)


def test_adjoint_identity(oracle_mod):
    """Re <A f, c> = <f, A^H c> on random f, c (explicit adjoint is the transpose)."""
    rng = np.random.default_rng(5)
    n, delta = 24, 9 * synth.ARCSEC
    f = rng.standard_normal((n, n))
    uv = _rand_uv(rng, 300, delta)
    c = rng.standard_normal(300) + 1j * rng.standard_normal(300)
    lhs = np.sum(np.conj(oracle_mod.dft_forward(f, uv, delta)) * c).real
    rhs = np.sum(f * oracle_mod.dft_adjoint(c, uv, delta, n))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.abs(f).sum() * np.abs(c).sum())


def test_dft_adjoint_pixels_matches_the_full_adjoint(oracle_mod):
    """O5 at selected pixels equals the whole-image adjoint at those pixels (corners, the
    phase centre and random interior pixels of a 16 x 16 grid, uv beyond Nyquist)."""
    rng = np.random.default_rng(16)
    n, delta = 16, 8 * synth.ARCSEC
    uv = _rand_uv(rng, 50, delta)
    c = rng.standard_normal(50) + 1j * rng.standard_normal(50)
    full = oracle_mod.dft_adjoint(c, uv, delta, n)
    pix = np.array([[0, 0], [0, n - 1], [n - 1, 0], [n - 1, n - 1], [n // 2, n // 2], [3, 11], [11, 3]]
                   + [list(rng.integers(0, n, 2)) for _ in range(9)])
    got = oracle_mod.dft_adjoint_pixels(c, uv, delta, n, pix)
    np.testing.assert_allclose(got, full[pix[:, 0], pix[:, 1]], rtol=0, atol=1e-12)


def test_dft_adjoint_pixels_brute_force_tiny(oracle_mod):
    """Every pixel of a 4 x 4 sub-image from pure-Python exponentials of the full phase
    (row index a pairs with v, column index b with u; sign +)."""
    n, delta = 4, 12 * synth.ARCSEC
    uv = np.array([[1234.5, -987.25], [-40000.0, 51234.0], [0.0, 77.0]])
    coef = np.array([0.3 - 1.1j, 2.0 + 0.5j, -0.7 + 0.25j])
    pix = np.array([[a, b] for a in range(n) for b in range(n)])
    want = []
    for a, b in pix:
        l, m = (b - n / 2) * delta, (a - n / 2) * delta
        want.append(sum((cc * cmath.exp(2j * math.pi * (u * l + v * m))).real for cc, (u, v) in zip(coef, uv)))
    got = oracle_mod.dft_adjoint_pixels(coef, uv, delta, n, pix)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)


# ----------------------------------------------------------------------------- O1 / O6

def test_reproject_integer_translation_is_crop(oracle_mod):
    rng = np.random.default_rng(6)
    sky = rng.standard_normal((40, 40))
    g = synth.identity_interp(16, row0=5, col0=9)
    np.testing.assert_array_equal(oracle_mod.reproject(sky, g), sky[5:21, 9:25])


def test_reproject_matches_scipy_linear(oracle_mod):
    """Library special case: bilinear with zero outside = map_coordinates(order=1,
    mode='constant') at interior fractional positions."""
    rng = np.random.default_rng(7)
    sky = rng.standard_normal((30, 30))
    g = rng.uniform(1.0, 27.5, size=(12, 12, 2))
    want = scipy.ndimage.map_coordinates(sky, [g[..., 0], g[..., 1]], order=1, mode="constant")
    np.testing.assert_allclose(oracle_mod.reproject(sky, g), want, rtol=0, atol=1e-12)


def test_reproject_partition_of_unity_and_outside(oracle_mod):
    rng = np.random.default_rng(8)
    n = 20
    g = rng.uniform(0.0, n - 1.0, size=(9, 9, 2))
    np.testing.assert_allclose(oracle_mod.reproject(np.full((n, n), 2.5), g), 2.5, atol=1e-13)
    far = np.full((3, 3, 2), -5.0)
    assert np.all(oracle_mod.reproject(np.ones((n, n)), far) == 0.0)
    # half a pixel beyond the last row: only the inside taps count
    edge = np.full((1, 1, 2), [n - 0.5, 3.0])
    assert oracle_mod.reproject(np.ones((n, n)), edge)[0, 0] == pytest.approx(0.5)


def test_reproject_adjoint_identity(oracle_mod):
    rng = np.random.default_rng(9)
    n = 25
    sky = rng.standard_normal((n, n))
    g = rng.uniform(-1.5, n + 0.5, size=(14, 14, 2))
    h = rng.standard_normal((14, 14))
    lhs = np.sum(oracle_mod.reproject(sky, g) * h)
    rhs = np.sum(sky * oracle_mod.reproject_adjoint(h, g, n))
    assert abs(lhs - rhs) < 1e-11


# ----------------------------------------------------------------------------- O7

def test_laplacian_kernel_is_the_papers(oracle_mod):
    d = _golden("laplacian_kernel.txt")
    delta = np.zeros((7, 7))
    delta[3, 3] = 1.0
    np.testing.assert_array_equal(oracle_mod.laplacian(delta)[2:5, 2:5], d)
    np.testing.assert_array_equal(oracle_mod.LAPLACIAN_KERNEL, d)


def test_laplacian_matches_convolve2d(oracle_mod):
    rng = np.random.default_rng(10)
    x = rng.standard_normal((17, 23))
    d = _golden("laplacian_kernel.txt")
    want = scipy.signal.convolve2d(x, d, mode="same", boundary="fill", fillvalue=0.0)
    np.testing.assert_allclose(oracle_mod.laplacian(x), want, rtol=0, atol=1e-12)


def test_laplacian_closed_forms(oracle_mod):
    n, c = 31, 1.7
    r, _ = oracle_mod.regulariser(np.full((n, n), c))
    assert r == pytest.approx(2.0 * c * c * (n + 2), rel=1e-14)
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    ramp = 0.3 * i - 1.2 * j + 4.0
    assert np.abs(oracle_mod.laplacian(ramp)[1:-1, 1:-1]).max() < 1e-12
    delta = np.zeros((11, 11))
    delta[5, 5] = 1.0
    _, grad = oracle_mod.regulariser(delta)
    np.testing.assert_allclose(grad[3:8, 3:8], _golden("biharmonic_stencil.txt"), atol=0)
    assert np.abs(grad).sum() == pytest.approx(np.abs(_golden("biharmonic_stencil.txt")).sum())


# ----------------------------------------------------------------------------- O8

def _sd_geom(n=128, sd_n=8, pix=30 * synth.ARCSEC, fwhm=4 * synth.ARCMIN):
    import oracle

    taps, rb = oracle.sd_beam_taps(fwhm, pix)
    stride = n // sd_n
    return oracle.sd_sampling_matrix(n, sd_n, stride, stride // 2, taps, rb), taps, rb, stride


def test_sd_constant_sky_is_preserved_away_from_edges(oracle_mod):
    G, taps, rb, stride = _sd_geom()
    assert taps.sum() == pytest.approx(1.0, abs=1e-15)
    t = oracle_mod.sd_forward(np.full((128, 128), 3.0), G)
    centres = stride // 2 + stride * np.arange(8)
    ok = (centres - rb >= 0) & (centres + rb < 128)
    np.testing.assert_allclose(t[np.ix_(ok, ok)], 3.0, rtol=1e-14)


def test_sd_delta_gives_sampled_gaussian(oracle_mod):
    pix, fwhm = 30 * synth.ARCSEC, 4 * synth.ARCMIN
    G, taps, rb, stride = _sd_geom(pix=pix, fwhm=fwhm)
    x = np.zeros((128, 128))
    x[40, 70] = 1.0
    t = oracle_mod.sd_forward(x, G)
    sig = fwhm / (2 * np.sqrt(2 * np.log(2)))
    norm = np.exp(-(np.arange(-rb, rb + 1) * pix) ** 2 / (2 * sig * sig)).sum()
    for p in range(8):
        for q in range(8):
            dy, dx = stride // 2 + p * stride - 40, stride // 2 + q * stride - 70
            want = 0.0
            if abs(dy) <= rb and abs(dx) <= rb:
                want = np.exp(-((dy * pix) ** 2 + (dx * pix) ** 2) / (2 * sig * sig)) / norm ** 2
            assert t[p, q] == pytest.approx(want, abs=1e-16)


def test_sd_adjoint_identity(oracle_mod):
    rng = np.random.default_rng(11)
    G, *_ = _sd_geom()
    x = rng.standard_normal((128, 128))
    e = rng.standard_normal((8, 8))
    lhs = np.sum(oracle_mod.sd_forward(x, G) * e)
    rhs = np.sum(x * oracle_mod.sd_adjoint(e, G))
    assert abs(lhs - rhs) < 1e-12 * np.abs(x).sum()


def test_sd_term_at_zero_sky_closed_form(oracle_mod):
    """K(0) = 1/2 sum T^2 / sigma_sd^2 and grad K(0) = -B^T S^T T / sigma_sd^2 (Sect. 2.4):
    the absolute scale of the fusion term, which a finite-difference test alone leaves free
    (a sigma vs sigma^2 slip in both K and its gradient would pass one)."""
    rng = np.random.default_rng(17)
    G, *_ = _sd_geom()
    t_map = rng.uniform(0.0, 5.0, size=(8, 8))
    for sigma in (0.37, 2.0):
        K, g = oracle_mod.sd_term(np.zeros((128, 128)), t_map, sigma, G)
        assert K == pytest.approx(0.5 * float(np.sum(t_map ** 2)) / sigma ** 2, rel=1e-14)
        # the gradient at zero pairs with the delta response: <e_ij, grad> = -sum T g g / s^2
        i, j = 40, 70
        want = -sum(t_map[p, q] * G[p, i] * G[q, j] for p in range(8) for q in range(8)) / sigma ** 2
        assert g[i, j] == pytest.approx(want, rel=1e-12, abs=1e-18)


# ----------------------------------------------------------------------------- O4 / O9

@pytest.fixture(scope="module")
def mini(oracle_mod):
    p = synth.config_c3_mini()
    oracle_mod.synthesize(p)
    return p


def test_adjoint_image_is_the_transpose_of_model_vis(oracle_mod, mini):
    """Re <model_vis(x), W v> = <x, adjoint_image(v)> over every pointing and channel of the
    overlapping mini mosaic (flagged entries carry garbage and must be skipped by both)."""
    rng = np.random.default_rng(18)
    x = rng.uniform(0, 50, size=mini.x_true.shape)
    v = rng.standard_normal(mini.n_vis) + 1j * rng.standard_normal(mini.n_vis)
    v[mini.flags == 1] = 1e30
    mv = oracle_mod.model_vis(mini, x)
    live = mini.flags == 0
    lhs = float(np.sum((np.conj(mv) * mini.weight * v)[live]).real)
    rhs = float(np.sum(x * oracle_mod.adjoint_image(mini, v)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_adjoint_image_of_the_data_is_minus_the_gradient_at_zero(oracle_mod, mini):
    """adjoint_image(y) = -grad Q(0) with lambda_r = lambda_s = 0 (Sect. 2.2: at x = 0 the
    residual is -y), the relation the dirty mosaic and the adjoint parity tests rely on."""
    import copy

    q = copy.copy(mini)
    q.lambda_r = q.lambda_s = 0.0
    _, g0 = oracle_mod.objective_grad(q, np.zeros_like(q.x_true))
    d = oracle_mod.adjoint_image(q, q.vis)
    np.testing.assert_allclose(d, -g0, rtol=0, atol=1e-12 * np.abs(g0).max())



def test_data_term_at_zero_sky(oracle_mod, mini):
    """J(0) = 1/2 sum w |y|^2 over live visibilities; flagged ones never count."""
    terms, _ = oracle_mod.objective_grad(mini, np.zeros_like(mini.x_true))
    live = mini.flags == 0
    y = mini.vis[live].astype(np.complex128)
    assert terms["Q"] == pytest.approx(0.5 * np.sum(mini.weight[live] * np.abs(y) ** 2), rel=1e-12)
    assert (mini.flags == 1).sum() > 0


def test_flagged_values_never_matter(oracle_mod, mini):
    rng = np.random.default_rng(12)
    x = rng.uniform(0, 50, size=mini.x_true.shape)
    t0, g0 = oracle_mod.objective_grad(mini, x)
    saved = mini.vis.copy()
    bad = mini.flags == 1
    mini.vis[bad] = 1e30 + 1e30j
    try:
        t1, g1 = oracle_mod.objective_grad(mini, x)
    finally:
        mini.vis[:] = saved
    assert t1["Q_tot"] == t0["Q_tot"]
    np.testing.assert_array_equal(g1, g0)


def test_noise_free_data_is_a_zero(oracle_mod):
    p = synth.config_c3_mini(seed=3102)
    p.noise[:] = 0
    oracle_mod.synthesize(p, with_sd=False)
    p.lambda_r = p.lambda_s = 0.0
    terms, g = oracle_mod.objective_grad(p, p.x_true)
    assert terms["Q"] < 1e-12 * 0.5 * np.sum(p.weight * np.abs(p.vis) ** 2)
    g0 = oracle_mod.objective_grad(p, np.zeros_like(p.x_true))[1]
    assert np.abs(g).max() < 1e-6 * np.abs(g0).max()


def test_hermitian_twin_doubles_the_data_term(oracle_mod):
    """Adding (-u, -v, conj y) for every visibility doubles J and its gradient for a real
    sky (the basis of folding u < 0 onto u > 0)."""
    p = synth.config_c1()
    p.lambda_r = 0.0
    oracle_mod.synthesize(p)
    rng = np.random.default_rng(13)
    x = rng.uniform(0, 1, size=p.x_true.shape)
    t1, g1 = oracle_mod.objective_grad(p, x)
    q = synth.config_c1()
    q.lambda_r = 0.0
    q.uv = np.concatenate([p.uv, -p.uv])
    q.vis = np.concatenate([p.vis, np.conj(p.vis)])
    q.weight = np.concatenate([p.weight, p.weight])
    q.vis_offsets = np.array([0, 2 * p.n_vis], dtype=np.int64)
    t2, g2 = oracle_mod.objective_grad(q, x)
    assert t2["Q"] == pytest.approx(2 * t1["Q"], rel=1e-12)
    np.testing.assert_allclose(g2, 2 * g1, rtol=1e-10, atol=1e-9 * np.abs(g1).max())


def test_permutation_invariance(oracle_mod):
    p = synth.config_c1()
    oracle_mod.synthesize(p)
    rng = np.random.default_rng(14)
    x = rng.uniform(0, 1, size=p.x_true.shape)
    t1, g1 = oracle_mod.objective_grad(p, x)
    perm = rng.permutation(p.n_vis)
    p.uv, p.vis, p.weight = p.uv[perm], p.vis[perm], p.weight[perm]
    t2, g2 = oracle_mod.objective_grad(p, x)
    assert t2["Q"] == pytest.approx(t1["Q"], rel=1e-12)
    np.testing.assert_allclose(g2, g1, rtol=1e-10, atol=1e-10 * np.abs(g1).max())


def test_gradient_matches_finite_differences(oracle_mod, mini):
    """Central differences of the FP64 objective (all terms on: data, Laplacian, single
    dish, overlapping pointings) on 64 random pixels.  Q_tot is quadratic in x, so the
    central difference has no truncation error and a large step only reduces rounding."""
    rng = np.random.default_rng(15)
    x = rng.uniform(0, 50, size=mini.x_true.shape)
    _, g = oracle_mod.objective_grad(mini, x)
    flat = x.reshape(-1)
    idx = rng.choice(flat.size, 64, replace=False)
    assert mini.lambda_r > 0 and mini.lambda_s > 0
    errs = []
    for i in idx:
        h = 0.5
        xp, xm = flat.copy(), flat.copy()
        xp[i] += h
        xm[i] -= h
        fp = oracle_mod.objective_grad(mini, xp.reshape(x.shape))[0]["Q_tot"]
        fm = oracle_mod.objective_grad(mini, xm.reshape(x.shape))[0]["Q_tot"]
        fd = (fp - fm) / (2 * h)
        errs.append(abs(fd - g.reshape(-1)[i]) / max(abs(g.reshape(-1)[i]), 1e-3 * np.abs(g).max()))
    assert max(errs) < 1e-7, max(errs)


def test_point_source_flux_recovery_without_regulariser(oracle_mod):
    """The paper's point-source validation (Sect. 4.1): with lambda_r = lambda_s = 0 and the
    positivity bound, L-BFGS-B on the FP64 objective puts each source's flux back on its
    pixel.  Bound: 3 sigma with sigma = 4 / sqrt(sum w s^2 A^2) (one-pixel curvature of
    the data term, inflated for the coupling between free pixels); statistical, so parity
    is unpinned beyond it."""
    import scipy.optimize

    p = oracle_mod.synthesize(synth.config_c1())
    n = p.x_true.size

    def f(x):
        t, g = oracle_mod.objective_grad(p, x.reshape(p.x_true.shape))
        return t["Q_tot"], g.ravel()

    r = scipy.optimize.minimize(f, np.zeros(n), jac=True, method="L-BFGS-B",
                                bounds=scipy.optimize.Bounds(np.zeros(n), np.full(n, np.inf)),
                                options={"maxiter": 1500, "ftol": 1e-14, "gtol": 1e-10})
    x = r.x.reshape(p.x_true.shape)[0]
    w = p.weight.astype(np.float64)
    for a, b in np.argwhere(p.x_true[0] > 0):
        A = float(p.beams[0][a, b])
        sigma = 4.0 / np.sqrt(np.sum(w) * (p.flux_scale[0] * A) ** 2)
        assert abs(x[a - 1:a + 2, b - 1:b + 2].sum() - p.x_true[0, a, b]) <= 3 * sigma
    assert x.min() >= 0.0


# ----------------------------------------------------------------------------- spectral term

def test_spectral_term_closed_forms(oracle_mod):
    """R_nu = 1/2 sum_c ||x_{c+1} - x_c||^2: zero on a channel-constant cube, 1/2 (C-1) N^2 s^2
    on a ramp x_c = c s with gradient -s / 0 / +s on the first / inner / last channels, and a
    delta in one channel gives value d^2 and gradient 2d, -d, -d (one-sided at the ends)."""
    rng = np.random.default_rng(60)
    C, N = 5, 6
    flat = np.repeat(rng.standard_normal((1, N, N)), C, axis=0)
    v, g = oracle_mod.spectral_term(flat)
    assert v == 0.0 and np.all(g == 0.0)
    s = 0.75
    ramp = np.repeat((np.arange(C) * s)[:, None, None], N, axis=1).repeat(N, axis=2)
    v, g = oracle_mod.spectral_term(ramp)
    assert v == pytest.approx(0.5 * (C - 1) * N * N * s * s, rel=1e-15)
    np.testing.assert_allclose(g[0], -s)
    np.testing.assert_allclose(g[1:-1], 0.0, atol=1e-15)
    np.testing.assert_allclose(g[-1], s)
    d = 1.3
    for c0, want in ((2, (2 * d, -d, -d)), (0, (d, None, -d)), (C - 1, (d, -d, None))):
        x = np.zeros((C, N, N))
        x[c0, 2, 3] = d
        v, g = oracle_mod.spectral_term(x)
        assert v == pytest.approx((1.0 if c0 in (0, C - 1) else 2.0) * 0.5 * d * d, rel=1e-15)
        assert g[c0, 2, 3] == pytest.approx(want[0])
        if want[1] is not None:
            assert g[c0 - 1, 2, 3] == pytest.approx(want[1])
        if want[2] is not None:
            assert g[c0 + 1, 2, 3] == pytest.approx(want[2])
        assert np.count_nonzero(g) == (3 if c0 not in (0, C - 1) else 2)
    assert oracle_mod.spectral_term(rng.standard_normal((1, N, N)))[0] == 0.0


def test_objective_with_spectral_term_matches_finite_differences(oracle_mod):
    """The full objective of a 4-channel mosaic with the spectral term on: central differences
    (exact for a quadratic) at pixels of the first, an inner and the last channel."""
    p = synth.config_c4_mini()
    e = p.expand()
    e.vis = p.vis
    e.lambda_nu = 0.37
    synth.attach_sd(e, oracle_mod.sd_model(e, e.x_true))
    rng = np.random.default_rng(61)
    x = rng.uniform(0, 50, size=e.x_true.shape)
    t, g = oracle_mod.objective_grad(e, x)
    assert t["Nu"] > 0 and t["Q_tot"] == pytest.approx(t["Q"] + e.lambda_s * t["K"] + e.lambda_r * t["R"]
                                                        + e.lambda_nu * t["Nu"], rel=1e-15)
    worst = 0.0
    for c in (0, 1, e.n_chan - 1):
        for _ in range(2):
            i, j = rng.integers(0, e.n_sky, 2)
            h = 0.5
            xp, xm = x.copy(), x.copy()
            xp[c, i, j] += h
            xm[c, i, j] -= h
            fd = (oracle_mod.objective_grad(e, xp)[0]["Q_tot"] - oracle_mod.objective_grad(e, xm)[0]["Q_tot"]) / (2 * h)
            worst = max(worst, abs(fd - g[c, i, j]) / max(abs(g[c, i, j]), 1e-3 * np.abs(g).max()))
    assert worst < 1e-7, worst
