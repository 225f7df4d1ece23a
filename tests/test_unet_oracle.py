"""Pins of the FP64 warm-start network layer oracle (CPU): closed forms, library special
cases, adjoint identities and finite differences."""
import numpy as np
import pytest
import scipy.signal

from oracle import unet as U


def test_bf16_rounding_known_values():
    x = np.array([1.0, 1.00390625, 1.0 + 2 ** -8 + 2 ** -10, 3.14159265, -2.5, 65504.0], dtype=np.float32)
    r = U.bf16(x)
    assert r[0] == 1.0
    assert r[1] == 1.0                    # 1 + 2^-8 is a tie: rounds to even (1.0)
    assert r[2] == 1.0 + 2 ** -7          # above the tie: rounds up
    assert r[3] == 3.140625
    assert r[4] == -2.5
    assert r[5] == 65536.0


def test_conv3x3_matches_correlate2d():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 7, 9, 3))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = U.conv3x3(x, w, b)
    for n in range(2):
        for o in range(4):
            want = b[o] + sum(scipy.signal.correlate2d(x[n, :, :, c], w[o, :, :, c], mode="same")
                              for c in range(3))
            np.testing.assert_allclose(y[n, :, :, o], want, atol=1e-12)


def test_conv3x3_delta_kernel_is_a_shift():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((1, 6, 6, 2))
    w = np.zeros((2, 3, 3, 2))
    w[0, 0, 2, 0] = 1.0  # reads x[i-1, j+1]
    w[1, 1, 1, 1] = 1.0  # identity on channel 1
    y = U.conv3x3(x, w)
    np.testing.assert_array_equal(y[0, 1:, :-1, 0], x[0, :-1, 1:, 0])
    assert np.all(y[0, 0, :, 0] == 0) and np.all(y[0, :, -1, 0] == 0)
    np.testing.assert_array_equal(y[..., 1], x[..., 1])


def test_conv3x3_grads_adjoint_and_fd():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 5, 6, 3))
    w = rng.standard_normal((4, 3, 3, 3))
    dy = rng.standard_normal((2, 5, 6, 4))
    lhs = np.sum(U.conv3x3(x, w) * dy)
    assert lhs == pytest.approx(np.sum(x * U.conv3x3_grad_input(dy, w, x.shape)), rel=1e-12)
    dw, db = U.conv3x3_grad_weight(x, dy)
    assert lhs == pytest.approx(np.sum(w * dw), rel=1e-12)
    b = rng.standard_normal(4)
    assert np.sum(U.conv3x3(x, w, b) * dy) - lhs == pytest.approx(np.sum(b * db), rel=1e-12)


def test_pool_and_up_adjoints():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 6, 8, 3))
    dy = rng.standard_normal((2, 3, 4, 3))
    # max pool is piecewise linear: its gradient is the transpose of the selection
    assert np.sum(U.maxpool2(x) * dy) == pytest.approx(np.sum(x * U.maxpool2_grad(x, dy)), rel=1e-12)
    u = rng.standard_normal((2, 3, 4, 3))
    du = rng.standard_normal((2, 6, 8, 3))
    assert np.sum(U.up2(u) * du) == pytest.approx(np.sum(u * U.up2_grad(du)), rel=1e-12)
    # ties go to the first position only
    t = np.ones((1, 2, 2, 1))
    g = U.maxpool2_grad(t, np.ones((1, 1, 1, 1)))
    assert g[0, 0, 0, 0] == 1 and g.sum() == 1


def test_maxpool2_forward_values_explicit_loop():
    """Forward values of the 2 x 2 max pool against an explicit loop over every window
    (negative values included, so a pool of |x| or a sum would fail)."""
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2, 6, 8, 3)) - 0.5
    y = U.maxpool2(x)
    assert y.shape == (2, 3, 4, 3)
    for n in range(2):
        for i in range(3):
            for j in range(4):
                for c in range(3):
                    want = max(x[n, 2 * i, 2 * j, c], x[n, 2 * i, 2 * j + 1, c],
                               x[n, 2 * i + 1, 2 * j, c], x[n, 2 * i + 1, 2 * j + 1, c])
                    assert y[n, i, j, c] == want


def test_adam_first_step_is_signed_lr():
    p = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -4.0, 1e-3])
    p1, m, v = U.adam(p, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    np.testing.assert_allclose(p1, p - 0.01 * np.sign(g), rtol=1e-5)


def test_network_gradient_matches_finite_differences():
    """End-to-end: the FP64 reverse pass composed from the layer gradients agrees with
    central differences of the composed network on random parameters."""
    rng = np.random.default_rng(4)
    levels, base, in_ch = 3, 4, 4
    shapes = U.unet_param_shapes(levels, base, in_ch)
    nparam = sum(int(np.prod(s)) if s else 1 for _, s in shapes)
    flat = rng.standard_normal(nparam) * 0.3
    x = rng.standard_normal((2, 8, 8, in_ch))
    t = rng.standard_normal((2, 8, 8))
    loss, g = U.unet_loss_grad(x, t, flat, levels, base, in_ch)
    assert loss == pytest.approx(U.unet_loss(x, t, flat, levels, base, in_ch), rel=1e-14)
    idx = rng.choice(nparam, 40, replace=False)
    for i in idx:
        e = np.zeros(nparam)
        e[i] = 1e-6
        fd = (U.unet_loss(x, t, flat + e, levels, base, in_ch) - U.unet_loss(x, t, flat - e, levels, base, in_ch)) / 2e-6
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])
