"""Full-size mosaic parity (GPU): 36 pointings on a 1024^2 sky, 384^2 sub-images, uneven
flagged visibility counts (about 34 M live of 39 M), single-dish map, lambda_r = 1e-2,
lambda_s = 1 — every (pointing, tile) work item of an evaluation batched into one launch
per stage.

Checked against the FP64 oracle on outputs it can compute one by one: sampled model
visibilities (direct DFT of the reprojected, beam-weighted sky of their pointing), the
objective at zero (closed form), the gradient at zero on sampled sky pixels (direct
adjoint sums over every visibility of every pointing that sees the pixel, the exact
bilinear transpose, and the single-dish gradient), plus the adjoint identity at full size.
Data: unit-variance complex noise (the model of the full problem is not needed)."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2609_17636_amd import Plan  # noqa: E402


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


@pytest.fixture(scope="module")
def c3():
    p = synth.config_c3()
    p.vis = p.noise.astype(np.complex64)
    p.weight = np.ones(p.n_vis, dtype=np.float32)
    synth.attach_sd(p, oracle.sd_model(p, p.x_true))
    return p


@pytest.fixture(scope="module")
def plan(c3):
    pl = Plan.from_problem(c3)
    pl.set_problem_data(c3)
    pl.autotune(1000.0)
    print("plan", pl.info(), flush=True)
    return pl


def _live_indices(p, rng, count):
    live = np.flatnonzero(p.flags == 0)
    return np.sort(rng.choice(live, count, replace=False))


def test_c3_forward_sampled(c3, plan):
    x = c3.x_true
    got = plan.forward(torch.tensor(x, dtype=torch.float32, device="cuda")).double().cpu().numpy()
    rng = np.random.default_rng(31)
    idx = _live_indices(c3, rng, 600)
    blocks = np.searchsorted(c3.vis_offsets, idx, side="right") - 1
    want = np.empty(idx.size, dtype=np.complex128)
    for k in np.unique(blocks):
        sel = blocks == k
        f = oracle.beam_weighted_subimage(c3, x[0], int(k), 0)
        want[sel] = oracle.dft_forward(f, c3.uv[idx[sel]], c3.pixel_rad)
    e = rel(got[idx, 0] + 1j * got[idx, 1], want)
    print(f"[c3 forward sampled] rel {e:.2e} over {np.unique(blocks).size} pointings", flush=True)
    assert e <= 1e-5
    flagged = np.flatnonzero(c3.flags != 0)[:1000]
    assert np.all(got[flagged] == 0.0)


def test_c3_objective_and_gradient_at_zero(c3, plan):
    zero = torch.zeros((1, 1024, 1024), dtype=torch.float32, device="cuda")
    terms, grad = plan.objective_grad(zero)
    grad = grad.double().cpu().numpy()[0]
    live = c3.flags == 0
    y = c3.vis.astype(np.complex128)
    q0 = 0.5 * float(np.sum(np.abs(y[live]) ** 2))
    G = oracle.sd_matrix_for(c3)
    k0, gsd = oracle.sd_term(np.zeros((1024, 1024)), c3.sd_map[0], c3.sd_sigma, G)
    print(f"[c3 Q(0)] Q {terms[1]:.9e} vs {q0:.9e}, K {terms[2]:.9e} vs {k0:.9e}", flush=True)
    assert abs(terms[1] - q0) <= 1e-6 * q0
    assert abs(terms[2] - k0) <= 1e-5 * k0
    assert abs(terms[0] - (q0 + c3.lambda_s * k0)) <= 1e-6 * terms[0]
    # sampled pixels, inside the mosaic footprint
    rng = np.random.default_rng(32)
    pix = rng.integers(200, 824, size=(12, 2))
    want = c3.lambda_s * gsd[pix[:, 0], pix[:, 1]]
    n_sub = c3.n_sub
    for k in range(c3.n_point):
        grid = c3.interp[k].astype(np.float64)
        s = slice(int(c3.vis_offsets[k]), int(c3.vis_offsets[k + 1]))
        lv = c3.flags[s] == 0
        coef = y[s][lv] * c3.weight[s][lv]
        uv = c3.uv[s][lv]
        for t, (i, j) in enumerate(pix):
            near = np.argwhere((np.abs(grid[..., 0] - i) < 1.5) & (np.abs(grid[..., 1] - j) < 1.5))
            if near.size == 0:
                continue
            adj = oracle.dft_adjoint_pixels(coef, uv, c3.pixel_rad, n_sub, near)
            gp = np.zeros((n_sub, n_sub))
            gp[near[:, 0], near[:, 1]] = -c3.flux_scale[0] * c3.beams[k][near[:, 0], near[:, 1]] * adj
            want[t] += oracle.reproject_adjoint(gp, grid, 1024)[i, j]
    got = grad[pix[:, 0], pix[:, 1]]
    e = rel(got, want)
    print(f"[c3 grad(0) sampled] rel {e:.2e}", flush=True)
    assert e <= 1e-5


def test_c3_adjoint_identity(c3, plan):
    rng = np.random.default_rng(33)
    x = rng.standard_normal((1, 1024, 1024)).astype(np.float32)
    v = rng.standard_normal((c3.n_vis, 2)).astype(np.float32)
    v[c3.flags != 0] = 0.0
    Ax = plan.forward(torch.tensor(x, device="cuda")).double().cpu().numpy()
    AHv = plan.adjoint(torch.tensor(v, device="cuda")).double().cpu().numpy()
    lhs = float(np.sum(Ax * v))
    rhs = float(np.sum(x * AHv))
    assert abs(lhs - rhs) <= 1e-4 * np.sqrt(np.sum(Ax ** 2) * np.sum(v.astype(np.float64) ** 2))


def _quadratic_identity(plan, x, label):
    """Q_tot is quadratic in x, so Q(x) - Q(0) = 1/2 <x, G(x) + G(0)> exactly, whatever the
    data: a property of the objective mode at a non-zero sky that holds at any size.  With
    Q(0) and G(0) pinned against the oracle and the forward pinned on sampled visibilities,
    a degrid that disagreed with its spread would break it."""
    zero = torch.zeros_like(x)
    t0, g0 = plan.objective_grad(zero)
    g0 = g0.double()
    t1, g1 = plan.objective_grad(x)
    xd = x.double()
    lhs = t1[0] - t0[0]
    rhs = 0.5 * float(torch.sum(xd * (g1.double() + g0)).item())
    print(f"[{label} quadratic identity] Q(x)-Q(0) {lhs:.9e} vs 1/2<x,G(x)+G(0)> {rhs:.9e} "
          f"rel {abs(lhs - rhs) / (abs(t1[0]) + abs(t0[0])):.2e}", flush=True)
    assert abs(lhs - rhs) <= 1e-5 * (abs(t1[0]) + abs(t0[0]))


def test_c3_objective_mode_at_a_nonzero_sky(c3, plan):
    """The autotuned mosaic launch (7-waves-per-SIMD build above 32,768 work items) at a
    uniform 0-50 K sky."""
    assert plan.info()["n_work_items"] >= 32768
    gen = torch.Generator(device="cuda").manual_seed(3)
    x = torch.rand((c3.n_chan, c3.n_sky, c3.n_sky), generator=gen, device="cuda") * 50.0
    _quadratic_identity(plan, x, "c3")
