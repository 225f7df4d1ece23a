"""Warm-start network kernels against the FP64 layer oracle (GPU).

Every 3x3 convolution consumes bf16 operands on the matrix cores and sums in FP32, so the
single-layer checks feed the oracle the same bf16-rounded operands and bound the
difference by the FP32 summation error gamma_K * sum|terms| (K = number of products per
output, u = 2^-24).  Pooling, upsampling, flips and the bf16 rounding itself are exact.

Through the whole network the two sides round their own activations to bf16 before every
convolution; an activation that lies within FP32 error of a bf16 rounding boundary can
round the other way, which moves that operand by one bf16 ulp (2^-8 relative).  The
network-level tolerances below are set from that: relative L2 differences of 1e-2 or less,
well under the 2^-8 that a systematic error in any layer would produce, and far below the
O(1) error of a wrong index, sign or operand.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import unet as U  # noqa: E402

pytestmark = pytest.mark.gpu

U24 = 2.0 ** -24


@pytest.fixture(scope="module")
def nn():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_17636_amd import unet

    return unet


def _bits_to_f64(bits):
    b = np.asarray(bits).astype(np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _wbits(nn, w):
    return nn.to_bf16(_dev(w))


def test_to_bf16_rounds_to_nearest_even(nn):
    rng = np.random.default_rng(10)
    x = np.concatenate([rng.standard_normal(5000) * 10 ** rng.uniform(-6, 6, 5000),
                        np.array([1.0, 1.00390625, 1.0 + 2 ** -8 + 2 ** -10, -2.5, 65504.0, 0.0, -0.0])])
    x = x.astype(np.float32)
    got = _bits_to_f64(nn.to_bf16(_dev(x)).cpu().numpy())
    np.testing.assert_array_equal(got, U.bf16(x))


@pytest.mark.parametrize("cin,cout,relu", [(4, 16, False), (8, 32, True), (12, 48, True), (16, 64, False),
                                           (20, 128, True), (24, 96, False), (64, 32, True), (32, 64, True),
                                           (96, 128, False)])
def test_conv3x3_matches_oracle(nn, cin, cout, relu):
    rng = np.random.default_rng(cin * 100 + cout)
    n, h, w = 2, 11, 19          # 418 pixels: six full 64-pixel blocks and a ragged one
    x = rng.standard_normal((n, h, w, cin)).astype(np.float32)
    wt = (rng.standard_normal((cout, 3, 3, cin)) * 0.3).astype(np.float32)
    b = rng.standard_normal(cout).astype(np.float32)
    y = nn.conv3x3(_dev(x), _wbits(nn, wt), bias=_dev(b), relu=relu).cpu().numpy()
    qx, qw = U.bf16(x), U.bf16(wt)
    want = U.conv3x3(qx, qw, b, relu=relu)
    bound = 9 * cin * U24 * (U.conv3x3(np.abs(qx), np.abs(qw)) + np.abs(b)) + 1e-30
    err = np.abs(y - want)
    assert np.all(err <= bound), (err.max(), bound[err > bound][:4])
    assert np.abs(want).max() > 1.0


@pytest.mark.parametrize("cin", [8, 32])
def test_conv3x3_mask_and_accumulate(nn, cin):
    rng = np.random.default_rng(11 + cin)
    n, h, w, cout = 1, 9, 13, 32
    x = rng.standard_normal((n, h, w, cin)).astype(np.float32)
    wt = rng.standard_normal((cout, 3, 3, cin)).astype(np.float32)
    mask = np.maximum(rng.standard_normal((n, h, w, cout)), 0).astype(np.float32)
    y0 = rng.standard_normal((n, h, w, cout)).astype(np.float32)
    out = _dev(y0)
    nn.conv3x3(_dev(x), _wbits(nn, wt), mask=_dev(mask), accumulate=True, out=out)
    qx, qw = U.bf16(x), U.bf16(wt)
    want = y0 + U.conv3x3(qx, qw) * (mask > 0)
    bound = 9 * cin * U24 * U.conv3x3(np.abs(qx), np.abs(qw)) + 2 * U24 * np.abs(want) + 1e-30
    assert np.all(np.abs(out.cpu().numpy() - want) <= bound)


def test_flip_gives_the_transposed_correlation(nn):
    rng = np.random.default_rng(12)
    cin, cout = 48, 32
    wt = rng.standard_normal((cout, 3, 3, cin)).astype(np.float32)
    bits = _wbits(nn, wt)
    fl = nn.conv3x3_flip(bits).cpu().numpy()
    want = np.transpose(bits.cpu().numpy()[:, ::-1, ::-1, :], (3, 1, 2, 0))
    np.testing.assert_array_equal(fl, want)
    # the convolution with flipped weights is the input gradient of the original one
    n, h, w = 2, 8, 10
    dy = rng.standard_normal((n, h, w, cout)).astype(np.float32)
    gin = nn.conv3x3(_dev(dy), torch.from_numpy(fl).cuda()).cpu().numpy()
    qdy, qw = U.bf16(dy), _bits_to_f64(bits.cpu().numpy())
    want = U.conv3x3_grad_input(qdy, qw, (n, h, w, cin))
    bound = 9 * cout * U24 * U.conv3x3_grad_input(np.abs(qdy), np.abs(qw), (n, h, w, cin)) + 1e-30
    assert np.all(np.abs(gin - want) <= bound)


@pytest.mark.parametrize("n,h,w,cin,cout", [(1, 6, 10, 4, 16), (2, 23, 33, 16, 32), (3, 32, 32, 8, 80),
                                             (2, 40, 51, 96, 64), (1, 7, 9, 6, 16), (1, 9, 11, 8, 18)])
def test_conv3x3_grad_weight_matches_oracle(nn, n, h, w, cin, cout):
    rng = np.random.default_rng(n * 1000 + h)
    x = rng.standard_normal((n, h, w, cin)).astype(np.float32)
    dy = rng.standard_normal((n, h, w, cout)).astype(np.float32)
    dw, db = nn.conv3x3_grad_weight(_dev(x), _dev(dy))
    qx, qdy = U.bf16(x), U.bf16(dy)
    wdw, wdb = U.conv3x3_grad_weight(qx, qdy)
    adw, _ = U.conv3x3_grad_weight(np.abs(qx), np.abs(qdy))
    P = n * h * w
    assert np.all(np.abs(dw.cpu().numpy() - wdw) <= (P + 8) * U24 * adw + 1e-30)
    # the bias gradient sums the FP32 dy itself (no bf16 rounding)
    np.testing.assert_allclose(db.cpu().numpy(), dy.astype(np.float64).sum(axis=(0, 1, 2)),
                               atol=P * U24 * np.abs(dy).sum(axis=(0, 1, 2)).max())


def test_pool_and_upsampling_layers(nn):
    rng = np.random.default_rng(13)
    n, h, w, c = 2, 10, 14, 24
    # ReLU-like input with many exact zeros and repeated values: exercises the tie rule
    x = np.maximum(np.round(rng.standard_normal((n, h, w, c)) * 2) / 2, 0).astype(np.float32)
    dy = rng.standard_normal((n, h // 2, w // 2, c)).astype(np.float32)
    np.testing.assert_array_equal(nn.pool2(_dev(x)).cpu().numpy(), U.maxpool2(x))
    np.testing.assert_array_equal(nn.pool2_grad(_dev(x), _dev(dy)).cpu().numpy(), U.maxpool2_grad(x, dy))
    acc0 = rng.standard_normal(x.shape).astype(np.float32)
    acc = nn.pool2_grad(_dev(x), _dev(dy), accumulate_into=_dev(acc0)).cpu().numpy()
    np.testing.assert_allclose(acc, acc0 + U.maxpool2_grad(x, dy), rtol=2 * U24, atol=0)
    u = rng.standard_normal((n, h // 2, w // 2, c)).astype(np.float32)
    np.testing.assert_array_equal(nn.up2(_dev(u)).cpu().numpy(), U.up2(u))
    du = rng.standard_normal((n, h, w, c)).astype(np.float32)
    want = U.up2_grad(du)
    bound = 3 * U24 * U.up2_grad(np.abs(du))
    assert np.all(np.abs(nn.up2_grad(_dev(du)).cpu().numpy() - want) <= bound)


def _net_case(nn, levels=3, base=16, batch=2, h=32, w=48, seed=5):
    net = nn.UNet(levels=levels, base=base, max_batch=batch, height=h, width=w, seed=seed)
    rng = np.random.default_rng(seed)
    # biases are zero at initialisation: give them values so their paths are exercised
    p = net.get_params()
    shapes = U.unet_param_shapes(levels, base, 4)
    o = 0
    for name, shp in shapes:
        k = int(np.prod(shp)) if shp else 1
        if name.endswith(".b"):
            p[o:o + k] = rng.standard_normal(k) * 0.05
        o += k
    net.set_params(p)
    x = rng.random((batch, h, w)).astype(np.float32)
    t = rng.random((batch, h, w)).astype(np.float32)
    x4 = np.zeros((batch, h, w, 4))
    x4[..., 0] = x
    return net, p.astype(np.float64), x, x4, t


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def test_network_forward_matches_oracle(nn):
    levels, base = 3, 16
    net, p, x, x4, _ = _net_case(nn, levels, base)
    y = net.forward(_dev(x)).cpu().numpy()
    want, _ = U.unet_forward(x4, U.unpack(p, levels, base, 4), levels, round_bf16=True)
    exact, _ = U.unet_forward(x4, U.unpack(p, levels, base, 4), levels, round_bf16=False)
    print("forward rel vs bf16-rounded oracle", _rel(y, want), "vs unrounded", _rel(y, exact))
    assert _rel(y, want) <= 1e-2
    assert np.abs(y - want).max() <= 5e-2 * np.abs(want).max()


def test_network_gradient_matches_oracle(nn):
    levels, base = 3, 16
    net, p, x, x4, t = _net_case(nn, levels, base, seed=6)
    loss, g = net.loss_grad(_dev(x), _dev(t))
    wloss, wg = U.unet_loss_grad(x4, t, p, levels, base, 4, round_bf16=True)
    assert loss == pytest.approx(wloss, rel=2e-2)
    o = 0
    for name, shp in U.unet_param_shapes(levels, base, 4):
        k = int(np.prod(shp)) if shp else 1
        r = _rel(g[o:o + k], wg[o:o + k])
        print(name, r)
        assert r <= 2e-2, (name, r)
        o += k
    # fixed-order reductions: a second evaluation is bit-identical
    loss2, g2 = net.loss_grad(_dev(x), _dev(t))
    assert loss2 == loss and np.array_equal(g, g2)


def test_train_step_is_adam_on_the_gradient_and_reduces_the_loss(nn):
    levels, base = 3, 16
    net, p, x, x4, _ = _net_case(nn, levels, base, seed=7)
    t = x + 1.0      # a learnable target (the FP64 oracle run of this loop drops the loss ~50x)
    loss0, g = net.loss_grad(_dev(x), _dev(t))
    lr = 1e-3
    l_step = net.train_step(_dev(x), _dev(t), lr)
    assert l_step == loss0
    p1 = net.get_params().astype(np.float64)
    want, _, _ = U.adam(p, g.astype(np.float64), np.zeros_like(p), np.zeros_like(p), 1, lr)
    np.testing.assert_allclose(p1, want, rtol=0, atol=lr * 1e-3 + 4 * U24 * np.abs(p).max())
    losses = [net.train_step(_dev(x), _dev(t), lr) for _ in range(60)]
    print("loss", loss0, "->", losses[-1])
    assert losses[-1] < 0.2 * loss0


def test_bad_network_geometry_is_rejected(nn):
    from paper_2609_17636_amd import IvxError

    with pytest.raises(IvxError):
        nn.UNet(levels=4, base=16, height=36, width=64)     # 36 not divisible by 8
    with pytest.raises(IvxError):
        nn.UNet(levels=3, base=24, height=32, width=32)     # base not a multiple of 16
