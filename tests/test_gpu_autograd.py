"""The hand-written backward behind torch.autograd (GPU), checked against the FP64 oracle
and finite differences of the FP64 build.

Objective: forward = ivx_objective_forward (or the value-only ivx_objective when x needs no
gradient), backward = ivx_objective_backward scaled by grad_output.  ForwardModel: forward =
ivx_forward (sky -> model visibilities), backward = ivx_forward_adjoint (its unweighted
transpose).  The paper obtains these gradients by automatic differentiation (Sect. 3.4).
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2609_17636_amd as ivx  # noqa: E402
from paper_2609_17636_amd import IvxError, Plan  # noqa: E402

TOL = {"f32": 1e-5, "f64": 1e-10}


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


@pytest.fixture(scope="module")
def mini():
    return oracle.synthesize(synth.config_c3_mini())


def _plan(p, precision="f32", blocking=None):
    plan = Plan.from_problem(p, precision=precision)
    plan.set_problem_data(p)
    if blocking:
        plan.set_blocking(*blocking)
    return plan


@pytest.mark.parametrize("blocking", [None, (8, 1, 128, 64, 1)])
def test_objective_backward_matches_the_oracle_gradient(mini, blocking):
    """Objective.apply(x).backward() against oracle.objective_grad (data term over four
    overlapping pointings with flags, Laplacian and single-dish terms on), for the vector and
    the matrix-core gridder; and bit for bit the fused evaluation's gradient."""
    plan = _plan(mini, blocking=blocking)
    rng = np.random.default_rng(51)
    xh = rng.uniform(0, 50, size=mini.x_true.shape)
    want_t, want_g = oracle.objective_grad(mini, xh)
    x = torch.tensor(xh, dtype=torch.float32, device="cuda", requires_grad=True)
    q = ivx.Objective.apply(x, plan)
    q.backward()
    got = x.grad.double().cpu().numpy()
    rq = abs(q.item() - want_t["Q_tot"]) / want_t["Q_tot"]
    print(f"[autograd {blocking}] relQ {rq:.2e} relG {rel(got, want_g):.2e}", flush=True)
    assert rq <= TOL["f32"]
    assert rel(got, want_g) <= TOL["f32"]
    terms, grad = plan.objective_grad(x.detach())
    assert q.item() == terms[0]
    assert np.array_equal(got, grad.double().cpu().numpy())


def test_objective_scales_by_grad_output_and_value_only_path(mini):
    plan = _plan(mini)
    rng = np.random.default_rng(52)
    xh = rng.uniform(0, 50, size=mini.x_true.shape)
    x = torch.tensor(xh, dtype=torch.float32, device="cuda", requires_grad=True)
    (-2.5 * ivx.Objective.apply(x, plan)).backward()
    terms, grad = plan.objective_grad(x.detach())
    np.testing.assert_allclose(x.grad.cpu().numpy(), -2.5 * grad.cpu().numpy(), rtol=1e-6, atol=0)
    # no gradient wanted: the value-only evaluation (nothing spread), the same data term sums
    with torch.no_grad():
        q = ivx.Objective.apply(x, plan)
    assert q.item() == terms[0]
    t_val = plan.objective(x.detach())
    assert np.array_equal(t_val, terms)


def test_backward_needs_its_forward(mini):
    plan = _plan(mini)
    x = torch.rand(mini.x_true.shape, device="cuda") * 50
    plan.objective_forward(x)
    plan.forward(x)  # any other use of the plan's buffers in between
    with pytest.raises(IvxError) as ei:
        plan.objective_backward(x)
    assert ei.value.code == -5
    plan.objective_forward(x)
    plan.objective_backward(x)
    with pytest.raises(IvxError):  # one backward per forward
        plan.objective_backward(x)


def test_forward_model_vjp_matches_the_oracle_transpose(mini):
    """ForwardModel's backward is the unweighted transpose of the forward model: against
    oracle.adjoint_image(weighted=False) element by element, and the inner-product identity
    <g, V(x)> = <VJP(g), x> through torch.autograd."""
    plan = _plan(mini)
    rng = np.random.default_rng(53)
    g = rng.standard_normal((mini.n_vis, 2))
    g[mini.flags != 0] = 0.0
    x = torch.tensor(rng.uniform(0, 50, size=mini.x_true.shape), dtype=torch.float32, device="cuda",
                     requires_grad=True)
    v = ivx.ForwardModel.apply(x, plan)
    gt = torch.tensor(g, dtype=torch.float32, device="cuda")
    (v * gt).sum().backward()
    got = x.grad.double().cpu().numpy()
    want = oracle.adjoint_image(mini, g[:, 0] + 1j * g[:, 1], weighted=False)
    print(f"[forward-model vjp] rel {rel(got, want):.2e}", flush=True)
    assert rel(got, want) <= TOL["f32"]


def test_torch_composed_data_term_equals_the_fused_objective(mini):
    """1/2 sum w |ForwardModel(x) - y|^2 built from torch operations, differentiated by
    autograd through ForwardModel's backward, equals the fused objective's data term and its
    gradient (lambda_r = lambda_s = 0), FP64 build."""
    import copy

    q = copy.copy(mini)
    q.lambda_r = q.lambda_s = 0.0
    plan = _plan(q, "f64")
    rng = np.random.default_rng(54)
    x = torch.tensor(rng.uniform(0, 50, size=q.x_true.shape), dtype=torch.float64, device="cuda",
                     requires_grad=True)
    y = torch.tensor(np.stack([q.vis.real, q.vis.imag], axis=1), dtype=torch.float64, device="cuda")
    w = torch.tensor(q.weight * (q.flags == 0), dtype=torch.float64, device="cuda")
    v = ivx.ForwardModel.apply(x, plan)
    loss = 0.5 * (w[:, None] * (v - y) ** 2).sum()
    loss.backward()
    terms, grad = plan.objective_grad(x.detach())
    assert abs(loss.item() - terms[0]) <= 1e-10 * terms[0]
    assert rel(x.grad.cpu().numpy(), grad.cpu().numpy()) <= 1e-10


def test_objective_backward_matches_finite_differences_fp64(mini):
    """Directional central differences of Objective (FP64 build): Q_tot is quadratic, so
    (Q(x + h d) - Q(x - h d)) / 2h equals <grad, d> up to rounding, for random directions."""
    plan = _plan(mini, "f64")
    rng = np.random.default_rng(55)
    x = torch.tensor(rng.uniform(0, 50, size=mini.x_true.shape), dtype=torch.float64, device="cuda",
                     requires_grad=True)
    ivx.Objective.apply(x, plan).backward()
    g = x.grad.detach()
    worst = 0.0
    for k in range(4):
        d = torch.tensor(rng.standard_normal(mini.x_true.shape), dtype=torch.float64, device="cuda")
        h = 5.0  # no truncation error for a quadratic: a long step only shrinks the rounding
        with torch.no_grad():
            fp = ivx.Objective.apply(x.detach() + h * d, plan).item()
            fm = ivx.Objective.apply(x.detach() - h * d, plan).item()
        fd = (fp - fm) / (2 * h)
        an = float(torch.sum(g * d).item())
        worst = max(worst, abs(fd - an) / abs(an))
    print(f"[autograd fd fp64] worst rel {worst:.2e}", flush=True)
    assert worst <= 1e-8
