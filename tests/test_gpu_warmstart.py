"""Learned warm start on the warm-start mosaic (GPU), at a small scale.

* the device solver converges on the mosaic and time-to-tolerance reaches the target from
  both starts;
* a start at the converged solution itself reaches the tolerance at the first
  evaluation (the target bookkeeping of the measurement);
* training the network on a few cold solutions lowers its loss, and its warm start begins
  below the cold start's objective value Q_tot(0).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ws():
    from paper_2609_17636_amd import warmstart

    return warmstart


@pytest.fixture(scope="module")
def mosaic(ws):
    return ws.Mosaic(autotune_ms=0)


def test_cold_solve_converges_and_targets_are_met(ws, mosaic):
    m = mosaic
    m.simulate(ws.HELDOUT_BASE + 7)
    r = m.solve()
    assert r.message in ("pgtol", "ftol") and float(r.x.min()) >= 0.0
    # starting at the solution: the first evaluation already meets (1 + 1e-4) J*
    again = m.solve(x0=r.x, target=(1 + ws.TOL) * r.fun)
    assert again.reached_target and again.nfev == 1


def test_training_and_warm_start(ws, mosaic):
    from paper_2609_17636_amd.unet import UNet

    m = mosaic
    D, X, info = ws.cold_solves(m, list(range(12)), maxiter=300)
    assert all(i["nit"] == 300 or i["message"] in ("pgtol", "ftol") for i in info)
    net = UNet(levels=4, base=32, max_batch=4, height=256, width=256, seed=1)
    hist, best = ws.train(net, D[:10], X[:10], epochs=6, batch=4, lr=1e-3, Dv=D[10:], Xv=X[10:], val_every=2,
                          lr_final=1e-4)
    print("train mse", hist, "best", best)
    assert hist[-1] < 0.5 * hist[0]
    # the restored parameters are those of the selected epoch
    assert best is not None and best[1] in (2, 4, 6)
    assert abs(ws.mse(net, D[10:], X[10:], 4) - best[0]) <= 1e-6 * best[0]
    held = ws.HELDOUT_BASE + 3
    m.simulate(held)
    j = m.solve().fun
    row = ws.time_to_tolerance(m, net, held, j, x_mean=X.mean(dim=0, keepdim=True) * ws.PEAK_K)
    print(row)
    assert np.isfinite(row["cold_s"]) and np.isfinite(row["warm_s"]) and np.isfinite(row["mean_s"])
    assert np.isfinite(row["clamp_s"])
    assert row["q_warm_start"] < row["q_cold_start"]


def test_parallel_cold_solves_match_sequential(ws, mosaic):
    """Solver threads (own plan, solver and stream each) give the sequential results."""
    other = ws.Mosaic(autotune_ms=0, blocking=ws.blocking_of(mosaic))
    seeds = [21, 22, 23, 24, 25]
    D1, X1, i1 = ws.cold_solves(mosaic, seeds, maxiter=80)
    D2, X2, i2 = ws.cold_solves_parallel([mosaic, other], seeds, maxiter=80)
    assert torch.equal(D1, D2) and torch.equal(X1, X2)
    assert [r["fun"] for r in i1] == [r["fun"] for r in i2]


def test_learned_start_beats_the_cold_start(ws, mosaic):
    """The gain of the learned start, at a small scale: a network trained briefly on 96 cold
    solutions, then on 8 held-out fields the time and the evaluations to reach (1 + 1e-4) J*
    from the learned start against the cold start (x0 = 0), the order of the solves rotating
    from field to field.  The median learned start must need fewer evaluations and less time
    than the median cold start; the mean-image start (no learning) and the learned start
    clamped at 0 instead of floored are reported beside them."""
    from paper_2609_17636_amd.unet import UNet

    other = [ws.Mosaic(autotune_ms=0, blocking=ws.blocking_of(mosaic)) for _ in range(3)]
    D, X, info = ws.cold_solves_parallel([mosaic] + other, list(range(200, 296)), maxiter=400)
    net = UNet(levels=4, base=32, max_batch=16, height=256, width=256, seed=3)
    hist, best = ws.train(net, D[:88], X[:88], epochs=30, batch=16, lr=1e-3, Dv=D[88:], Xv=X[88:], val_every=5,
                          lr_final=1e-4)
    x_mean = X.mean(dim=0, keepdim=True) * ws.PEAK_K
    rows = []
    for i, seed in enumerate(range(ws.HELDOUT_BASE + 40, ws.HELDOUT_BASE + 48)):
        mosaic.simulate(seed)
        j_star = mosaic.solve().fun
        rows.append(ws.time_to_tolerance(mosaic, net, seed, j_star, x_mean=x_mean, order=i))
    s = ws.summarise(rows)
    print(f"[warm start] train mse {hist[0]:.4f} -> {hist[-1]:.4f}; cold {s['cold_s_median']:.3f} s / "
          f"{s['cold_nfev_median']:.0f} evals, learned {s['warm_s_median']:.3f} s / {s['warm_nfev_median']:.0f} evals, "
          f"mean image {s['mean_image_s_median']:.3f} s / {s['mean_image_nfev_median']:.0f} evals, "
          f"clamped learned {s['clamp_s_median']:.3f} s / {s['clamp_nfev_median']:.0f} evals; "
          f"ms per eval {s['ms_per_eval_median']}; learned faster on {s['warm_wins_fraction']:.2f}", flush=True)
    assert s["both_reached"] == len(rows)
    assert s["warm_nfev_median"] < s["cold_nfev_median"]
    assert s["warm_s_median"] < s["cold_s_median"]


def test_prefix_walk_gives_the_full_sort_iterates(ws, mosaic):
    """The Cauchy search sorts only the breakpoints below a sampled threshold first (an exact
    prefix of the full order) and all of them only when the minimiser lies beyond: the
    iterates are bitwise those of sorting every breakpoint every time, on 65,536 variables
    (tens of thousands of breakpoints per search), from a cold and from a flat start."""
    mosaic.simulate(ws.HELDOUT_BASE + 7)
    for x0 in (None, torch.full((1, mosaic.n, mosaic.n), 5.0, device="cuda")):
        a = mosaic.solve(x0=x0, maxiter=150)
        b = mosaic.solve(x0=x0, maxiter=150, full_sort=True)
        print(f"[prefix walk] walks {a.n_walks} (full sorts {a.n_walks_full}) vs {b.n_walks} ({b.n_walks_full}); "
              f"{1e3 * a.seconds / a.nfev:.3f} vs {1e3 * b.seconds / b.nfev:.3f} ms per evaluation", flush=True)
        assert (a.nit, a.nfev, a.fun, a.n_walks) == (b.nit, b.nfev, b.fun, b.n_walks)
        assert [f for _, f in a.history] == [f for _, f in b.history]
        assert torch.equal(a.x, b.x)
        assert b.n_walks_full == b.n_walks
        assert a.n_walks_full < a.n_walks / 4


def test_published_results_give_the_stream_wait_iterates(ws, mosaic):
    """The host reads each solver step's results as soon as the step's last kernel has
    published them (a sequence number in the mapped buffer) instead of after the stream has
    drained: bitwise the same iterates as waiting for the stream, on the same solve."""
    mosaic.simulate(ws.HELDOUT_BASE + 9)
    a = mosaic.solve(maxiter=120)
    b = mosaic.solve(maxiter=120, stream_wait=True)
    print(f"[published waits] {1e3 * a.seconds / a.nfev:.3f} vs {1e3 * b.seconds / b.nfev:.3f} ms per evaluation "
          f"(stream waits)", flush=True)
    assert (a.nit, a.nfev, a.fun, a.n_walks, a.n_walks_full) == (b.nit, b.nfev, b.fun, b.n_walks, b.n_walks_full)
    assert [f for _, f in a.history] == [f for _, f in b.history]
    assert torch.equal(a.x, b.x)
