"""Parity of the full forward model (Sect. 2.1, Eq. vis: the 1/n factor and the w (n - 1)
phase, w-stacked on the GPU) with the FP64 oracle's direct sums (GPU).

Wide-field single pointing (64^2 at 60 arcsec: the dropped phase reaches ~9 rad at the
corners on the longest baselines), the 2x2 SIN-grid mosaic with flags and the single-dish
term, and the shared-uv mini cube (w scaled per channel like uv): objective, gradient, model
visibilities and adjoint element by element, in the FP32 build (tolerance 1e-5 relative) and
the FP64 build (1e-10).  The coplanar model misses the full one by far more than the
tolerance on these problems, so the checks see the w term.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2609_17636_amd import IvxError, Plan  # noqa: E402

TOL = {"f32": 1e-5, "f64": 1e-10}
# the matrix-core gridder's w-plane modes (float build, windows of at most 16 x 16 cells)
MX = "matrix-core"


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


@pytest.fixture(scope="module")
def single():
    return oracle.synthesize(synth.config_w_single(), with_sd=False)


@pytest.fixture(scope="module")
def mosaic():
    return oracle.synthesize(synth.config_c3_mini(w_term=True))


@pytest.fixture(scope="module")
def cube():
    p = synth.config_c4_mini(w_term=True)
    e = p.expand()
    mv = oracle.model_vis(e, e.x_true)
    live = p.flags == 0
    sig = 0.01 * float(np.abs(mv[live]).max())
    p.vis = (mv + sig * p.vis.astype(np.complex128)).astype(np.complex64)
    p.weight[:] = 1.0 / sig ** 2
    synth.attach_sd(p, oracle.sd_model(e, p.x_true))
    return p


def _plan(p, precision, blocking=None, w=True, **kw):
    plan = Plan.from_problem(p, precision=precision, **kw)
    if hasattr(p, "pt_offsets"):
        plan.set_cube_data(p)
    else:
        plan.set_problem_data(p)
    if blocking == MX:
        # the matrix-core gridder: the largest tile whose window (T + W - 1) fits 16 cells
        plan.set_blocking(17 - plan.info()["kernel_width"], 1, 512, 64, 1)
    elif blocking is not None:
        plan.set_blocking(*blocking)
    if w:
        plan.set_w(p.w)
    return plan


def _eval(plan, x):
    sky = torch.tensor(np.asarray(x), dtype=plan.torch_dtype, device="cuda")
    terms, grad = plan.objective_grad(sky)
    torch.cuda.synchronize()
    return terms, grad.double().cpu().numpy()


def _check(p, e, plan, precision, label):
    """Q_tot, Q, K, R and the gradient (2-norm) at zero, at the true sky (gradient against the
    larger of its norm and the norm at zero: the residual there is noise) and at a random sky."""
    tol = TOL[precision]
    rng = np.random.default_rng(3)
    pts = {"zero": np.zeros_like(e.x_true), "true": e.x_true,
           "rand": rng.uniform(0.0, e.x_true.max(), size=e.x_true.shape)}
    g0 = None
    for name, x in pts.items():
        want_t, want_g = oracle.objective_grad(e, x)
        if name == "zero":
            g0 = np.linalg.norm(want_g)
        terms, grad = _eval(plan, x)
        print(f"[{label}/{precision}] x={name} Q_tot {terms[0]:.10e} oracle {want_t['Q_tot']:.10e} "
              f"relQ {abs(terms[0] - want_t['Q_tot']) / want_t['Q_tot']:.2e} relG {rel(grad, want_g):.2e}",
              flush=True)
        assert abs(terms[0] - want_t["Q_tot"]) <= tol * abs(want_t["Q_tot"]), (name, terms, want_t)
        assert abs(terms[1] - want_t["Q"]) <= tol * abs(want_t["Q_tot"])
        assert abs(terms[2] - want_t["K"]) <= tol * abs(want_t["Q_tot"]) + 1e-300
        assert abs(terms[3] - want_t["R"]) <= tol * max(abs(want_t["R"]), 1e-300) + 1e-300
        scale = max(np.linalg.norm(want_g), g0) if name == "true" else np.linalg.norm(want_g)
        assert np.linalg.norm(grad - want_g) <= tol * scale, name


@pytest.mark.parametrize("precision", ["f32", "f64"])
@pytest.mark.parametrize("blocking", [None, (8, 1, 256, 64, 1), (14, 1, 128, 16, 1)],
                         ids=["auto", "matrix-core-plan", "vector-plan"])
def test_single_pointing_objective(single, precision, blocking):
    if precision == "f64" and blocking is not None and blocking[3] == 64:
        pytest.skip("the matrix-core blocking is float only")
    plan = _plan(single, precision, blocking)
    info = plan.w_info()
    print(f"[w-single] {info}", flush=True)
    assert info["enabled"] and info["planes"] >= 10
    _check(single, single, plan, precision, "w-single")


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_single_pointing_forward_and_adjoint(single, precision):
    p = single
    plan = _plan(p, precision)
    tol = TOL[precision]
    sky = torch.tensor(p.x_true, dtype=plan.torch_dtype, device="cuda")
    got = plan.forward(sky).double().cpu().numpy()
    got = got[:, 0] + 1j * got[:, 1]
    want = oracle.model_vis(p, p.x_true)
    err = np.abs(got - want).max() / np.abs(want).max()
    print(f"[w-forward/{precision}] max err / max |V| {err:.2e}", flush=True)
    assert err <= tol
    rng = np.random.default_rng(5)
    y = rng.normal(size=p.n_vis) + 1j * rng.normal(size=p.n_vis)
    yt = torch.tensor(np.stack([y.real, y.imag], axis=1), dtype=plan.torch_dtype, device="cuda")
    adj = plan.adjoint(yt).double().cpu().numpy()
    want_a = oracle.adjoint_image(p, y)
    print(f"[w-adjoint/{precision}] rel {rel(adj, want_a):.2e}", flush=True)
    assert rel(adj, want_a) <= tol
    fa = plan.forward_adjoint(yt).double().cpu().numpy()
    assert rel(fa, oracle.adjoint_image(p, y, weighted=False)) <= tol


def test_the_w_term_is_visible_at_this_tolerance(single):
    """The coplanar model misses the full one by orders of magnitude more than 1e-5 here."""
    full, _ = oracle.objective_grad(single, single.x_true * 0.5)
    w = single.w
    single.w = None
    try:
        copl, _ = oracle.objective_grad(single, single.x_true * 0.5)
    finally:
        single.w = w
    assert abs(full["Q"] - copl["Q"]) > 1e3 * TOL["f32"] * full["Q"]


PLANS = [("f32", None), ("f64", None), ("f32", MX)]
PLAN_IDS = ["f32", "f64", "f32-matrix-core"]


@pytest.mark.parametrize("precision,blocking", PLANS, ids=PLAN_IDS)
def test_mosaic_objective(mosaic, precision, blocking):
    plan = _plan(mosaic, precision, blocking)
    print(f"[w-mosaic] {plan.w_info()} {plan.info()}", flush=True)
    _check(mosaic, mosaic, plan, precision, "w-mosaic")


@pytest.mark.parametrize("precision,blocking", PLANS, ids=PLAN_IDS)
def test_cube_objective_shared_uv(cube, precision, blocking):
    plan = _plan(cube, precision, blocking)
    print(f"[w-cube] {plan.w_info()}", flush=True)
    _check(cube, cube.expand(), plan, precision, "w-cube")


def test_matrix_core_forward_and_adjoint_on_the_mosaic(mosaic):
    """Model visibilities and the adjoint image of the w-plane modes on the matrix cores,
    element by element against the oracle's direct sums (blocks with flags, several
    pointings)."""
    p = mosaic
    plan = _plan(p, "f32", MX)
    assert plan.info()["lanes"] == 64
    sky = torch.tensor(p.x_true, dtype=plan.torch_dtype, device="cuda")
    got = plan.forward(sky).double().cpu().numpy()
    got = got[:, 0] + 1j * got[:, 1]
    want = oracle.model_vis(p, p.x_true)
    live = p.flags == 0
    err = np.abs(got[live] - want[live]).max() / np.abs(want[live]).max()
    print(f"[w-mx-forward] max err / max |V| {err:.2e}", flush=True)
    assert err <= TOL["f32"]
    rng = np.random.default_rng(8)
    y = (rng.normal(size=p.n_vis) + 1j * rng.normal(size=p.n_vis)) * live
    yt = torch.tensor(np.stack([y.real, y.imag], axis=1), dtype=plan.torch_dtype, device="cuda")
    adj = plan.adjoint(yt).double().cpu().numpy()
    want_a = oracle.adjoint_image(p, y)
    print(f"[w-mx-adjoint] rel {rel(adj, want_a):.2e}", flush=True)
    assert rel(adj, want_a) <= TOL["f32"]


def test_value_and_split_evaluations_agree(mosaic):
    plan = _plan(mosaic, "f64")
    sky = torch.tensor(mosaic.x_true * 0.7, dtype=plan.torch_dtype, device="cuda")
    t_full, g_full = plan.objective_grad(sky)
    g_full = g_full.cpu().numpy()
    t_val = plan.objective(sky)
    t_fwd = plan.objective_forward(sky)
    g_bwd = plan.objective_backward(sky, scale=2.0).cpu().numpy()
    np.testing.assert_allclose(t_val, t_full, rtol=1e-13)
    np.testing.assert_allclose(t_fwd, t_full, rtol=1e-13)
    np.testing.assert_allclose(g_bwd, 2.0 * g_full, rtol=1e-12, atol=1e-12 * np.abs(g_full).max())


def test_blocking_change_and_return_to_the_coplanar_model(mosaic):
    """A new blocking re-sorts the records: the full model follows it.  set_w(None) returns
    the plan to the coplanar model (checked against the oracle without w)."""
    plan = _plan(mosaic, "f32")
    plan.set_blocking(12, 2, 96, 16, 1)
    _check(mosaic, mosaic, plan, "f32", "w-mosaic-reblocked")
    plan.set_w(None)
    w = mosaic.w
    mosaic.w = None
    try:
        _check(mosaic, mosaic, plan, "f32", "coplanar-after-w")
    finally:
        mosaic.w = w


def test_bad_w_is_rejected(single):
    plan = _plan(single, "f32", w=False)
    bad = single.w.copy()
    bad[17] = np.nan
    with pytest.raises(IvxError) as e:
        plan.set_w(bad)
    assert "not finite" in str(e.value)
    with pytest.raises(IvxError):
        plan.set_w(single.w, w_width=1)
    # the plan keeps the coplanar model and still evaluates
    assert not plan.w_info()["enabled"]
    sky = torch.zeros((1, single.n_sky, single.n_sky), device="cuda")
    plan.objective_grad(sky)


def test_empty_and_fully_flagged_blocks():
    """A pointing whose every sample is flagged has no record and no w plane: its sub-image
    gradient must still be cleared, and the other pointings evaluate as usual."""
    import copy

    p = copy.deepcopy(synth.config_c3_mini(w_term=True))
    s = p.block(1, 0)
    p.flags[s] = 1
    oracle.synthesize(p)
    plan = _plan(p, "f64")
    info = plan.w_info()
    assert info["enabled"]
    _check(p, p, plan, "f64", "w-mosaic-flagged-block")
