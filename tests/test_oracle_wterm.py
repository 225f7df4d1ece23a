"""Pins of the oracle's full forward model (the 1/n factor and the w (n - 1) phase of Eq. vis,
Sect. 2.1) against closed forms, invariants, the coplanar special case and brute force (CPU
only).  Every pin is chosen so that a plausible slip fails it: n instead of 1/n, (1 - n)
instead of (n - 1), a dropped w factor, a swapped l/m axis, a conjugated adjoint."""
import cmath
import math

import numpy as np
import pytest

import synth


def _uvw(rng, m, delta, span=3.0, wmax=4000.0):
    uv = rng.uniform(-span, span, size=(m, 2)) / delta
    w = rng.uniform(-wmax, wmax, size=(m, 1))
    return np.concatenate([uv, w], axis=1)


def test_zero_w_is_the_coplanar_transform_of_f_over_n(oracle_mod):
    """w = 0 leaves the 1/n factor only: the full model equals the coplanar transform of
    f / n, with n = sqrt(1 - l^2 - m^2) formed here from its definition."""
    rng = np.random.default_rng(11)
    n, delta = 24, 0.01
    f = rng.uniform(0, 1, (n, n))
    uvw = _uvw(rng, 300, delta)
    uvw[:, 2] = 0.0
    c = n // 2
    l = (np.arange(n) - c) * delta
    nn = np.sqrt(1.0 - l[None, :] ** 2 - l[:, None] ** 2)
    ref = oracle_mod.dft_forward(f / nn, uvw[:, :2], delta)
    got = oracle_mod.dft_forward_w(f, uvw, delta)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-11 * np.abs(ref).max())


def test_phase_centre_source_is_flat_for_any_w(oracle_mod):
    """At l = m = 0, n = 1: the w phase vanishes and V_j = S for every (u, v, w)."""
    rng = np.random.default_rng(12)
    n, delta = 16, 0.02
    f = np.zeros((n, n))
    f[n // 2, n // 2] = 0.9
    v = oracle_mod.dft_forward_w(f, _uvw(rng, 400, delta, wmax=1e5), delta)
    np.testing.assert_allclose(v, 0.9, rtol=0, atol=1e-13)


@pytest.mark.parametrize("da,db,delta", [(0, 2, 0.3), (4, 3, 0.12), (3, 0, 0.2)])
def test_off_centre_source_with_exact_n(oracle_mod, da, db, delta):
    """A source at l = db delta, m = da delta with l^2 + m^2 = 0.36 has n = 0.8 exactly:
    V = S / 0.8 exp(-2 pi i (u l + v m - 0.2 w)).  Rows are m, columns are l; the image is
    just large enough to hold the source, so every pixel stays inside the unit circle."""
    l, m = db * delta, da * delta
    assert abs(l * l + m * m - 0.36) < 1e-12
    n = 2 * max(da, db) + 1
    c = n // 2
    f = np.zeros((n, n))
    f[c + da, c + db] = 1.3
    rng = np.random.default_rng(13)
    uvw = rng.uniform(-50, 50, size=(64, 3))
    got = oracle_mod.dft_forward_w(f, uvw, delta)
    ref = [1.3 / 0.8 * cmath.exp(-2j * math.pi * (u * l + v * m + w * (0.8 - 1.0))) for u, v, w in uvw]
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)


def test_hermitian_symmetry_in_all_three_coordinates(oracle_mod):
    """For a real image, V(-u, -v, -w) = conj V(u, v, w): the fold the gridder relies on."""
    rng = np.random.default_rng(14)
    n, delta = 20, 0.015
    f = rng.normal(size=(n, n))
    uvw = _uvw(rng, 200, delta)
    a = oracle_mod.dft_forward_w(f, uvw, delta)
    b = oracle_mod.dft_forward_w(f, -uvw, delta)
    np.testing.assert_allclose(b, np.conj(a), rtol=0, atol=1e-11 * np.abs(a).max())


def test_brute_force_tiny(oracle_mod):
    """4 x 4 image, 5 visibilities: the definition summed pixel by pixel in Python."""
    rng = np.random.default_rng(15)
    n, delta = 4, 0.05
    f = rng.normal(size=(n, n))
    uvw = _uvw(rng, 5, delta, wmax=300.0)
    got = oracle_mod.dft_forward_w(f, uvw, delta)
    for j, (u, v, w) in enumerate(uvw):
        s = 0j
        for a in range(n):
            for b in range(n):
                l, m = (b - n // 2) * delta, (a - n // 2) * delta
                nn = math.sqrt(1.0 - l * l - m * m)
                s += f[a, b] / nn * cmath.exp(-2j * math.pi * (u * l + v * m + w * (nn - 1.0)))
        assert abs(got[j] - s) < 1e-11, (j, got[j], s)


def test_adjoint_identity(oracle_mod):
    """Re <F_w f, c> = <f, F_w^T c> for real f and complex c."""
    rng = np.random.default_rng(16)
    n, delta = 18, 0.02
    f = rng.normal(size=(n, n))
    uvw = _uvw(rng, 150, delta)
    coef = rng.normal(size=150) + 1j * rng.normal(size=150)
    lhs = float(np.sum((oracle_mod.dft_forward_w(f, uvw, delta) * np.conj(coef)).real))
    rhs = float(np.sum(f * oracle_mod.dft_adjoint_w(coef, uvw, delta, n)))
    assert abs(lhs - rhs) < 1e-10 * max(1.0, abs(lhs)), (lhs, rhs)


def test_adjoint_pixels_match_the_full_adjoint_and_brute_force(oracle_mod):
    rng = np.random.default_rng(17)
    n, delta = 16, 0.025
    uvw = _uvw(rng, 90, delta)
    coef = rng.normal(size=90) + 1j * rng.normal(size=90)
    full = oracle_mod.dft_adjoint_w(coef, uvw, delta, n)
    pix = np.array([[0, 0], [3, 11], [8, 8], [15, 2], [15, 15]])
    got = oracle_mod.dft_adjoint_w_pixels(coef, uvw, delta, n, pix)
    np.testing.assert_allclose(got, full[pix[:, 0], pix[:, 1]], rtol=0, atol=1e-10)
    a, b = 3, 11
    l, m = (b - n // 2) * delta, (a - n // 2) * delta
    nn = math.sqrt(1 - l * l - m * m)
    s = sum((cj * cmath.exp(2j * math.pi * (u * l + v * m + w * (nn - 1)))).real
            for cj, (u, v, w) in zip(coef, uvw)) / nn
    assert abs(got[1] - s) < 1e-10


def test_small_angle_phase_error_is_pi_w_theta_squared(oracle_mod):
    """The phase the coplanar model drops for a source at distance r = sqrt(l^2 + m^2) from
    the phase centre is 2 pi w (1 - n) = pi w r^2 + pi w r^4 / 4 + ..., pi w r^2 to leading
    order (the error estimate of Sect. 2.1); checked for w = 10^4 and r from 5 to 40 arcmin,
    with |V| = 1 / n."""
    delta = 5 * synth.ARCMIN
    n = 32
    c = n // 2
    w = 1.0e4
    for k in (1, 2, 4, 8):
        f = np.zeros((n, n))
        f[c + k, c] = 1.0
        r = k * delta
        full = oracle_mod.dft_forward_w(f, np.array([[0.0, 0.0, w]]), delta)[0]
        assert abs(abs(full) - 1.0 / math.sqrt(1 - r * r)) < 1e-13
        dev = cmath.phase(full * cmath.exp(-1j * math.pi * w * r * r))  # small: no wrap
        assert 0.0 < dev < 1.01 * math.pi * w * r ** 4 / 4 + 1e-13, (k, dev)
        assert dev > 0.99 * math.pi * w * r ** 4 / 4


def test_objective_uses_the_full_model_when_w_is_present(oracle_mod):
    """With w attached the objective's data term and gradient follow the full model: the
    gradient matches central differences of the value, and dropping w changes the value."""
    p = synth.single_pointing("w-mini", 7, 16, 120.0, 4, 400, "diffuse", 0.0, ("abs", 0.05),
                              w_term=True)
    assert p.w is not None and np.abs(p.w).max() > 1000
    oracle_mod.synthesize(p, with_sd=False)
    rng = np.random.default_rng(18)
    x = rng.uniform(0, 20, size=(1, 16, 16))
    t, g = oracle_mod.objective_grad(p, x)
    h = 1e-3
    for (a, b) in [(2, 3), (8, 8), (13, 1)]:
        xp, xm = x.copy(), x.copy()
        xp[0, a, b] += h
        xm[0, a, b] -= h
        fd = (oracle_mod.objective_grad(p, xp)[0]["Q_tot"] - oracle_mod.objective_grad(p, xm)[0]["Q_tot"]) / (2 * h)
        assert abs(fd - g[0, a, b]) < 1e-6 * max(1.0, abs(fd)), (a, b, fd, g[0, a, b])
    w = p.w
    p.w = None
    t0, _ = oracle_mod.objective_grad(p, x)
    p.w = w
    assert abs(t0["Q"] - t["Q"]) > 1e-6 * t["Q"]


def test_generated_w_follows_the_baseline_geometry():
    """u^2 + v^2 + w^2 is the squared baseline length in wavelengths at every hour angle
    (the rotation preserves length; the array is planar, so the up component is 0), and
    the (u, v) columns are those of the coplanar generator."""
    rng = np.random.default_rng(19)
    bl = synth.baselines(synth.antenna_layout(rng, 12, 2000.0))
    uvw = synth.uvw_tracks(bl, 7, synth.LMC_DEC, 1.4e9)
    lam = synth.C_LIGHT / 1.4e9
    L = np.linalg.norm(bl, axis=1) / lam
    np.testing.assert_allclose(np.linalg.norm(uvw.reshape(7, -1, 3), axis=2), np.broadcast_to(L, (7, L.size)),
                               rtol=1e-12)
    np.testing.assert_array_equal(synth.uv_tracks(bl, 7, synth.LMC_DEC, 1.4e9), uvw[:, :2])
