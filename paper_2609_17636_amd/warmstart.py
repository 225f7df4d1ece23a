"""Learned warm start of the Classic3D solve, and its time-to-tolerance measurement.

The paper solves every field from the null prior x0 = 0 (Sect. 3.4).  Here a 4-level
U-Net (include/ivx_unet.h) maps the normalised dirty mosaic d = -grad Q_tot(0) / max|d|
to a first guess x0 = 50 K * max(net(d), 0), trained on converged cold-start solutions of
the same objective, and the solve starts from x0 instead.

Workload (warm-start mosaic): 256^2 sky at 30", 3 x 3 hexagonal mosaic of 20' Gaussian
beams at 40 px pitch, 128^2 sub-images, 200,000 visibilities per pointing (1.8 M),
lambda_r = 1e-2, no single-dish term.  Each field seed gives a k^-3 log-normal sky
(0-50 K); its visibilities are the FP64 HIP forward of that sky plus complex Gaussian noise
of 1% of the peak model amplitude per pointing (natural weights), the noise drawn from a
device generator seeded with the field seed.

Time-to-tolerance: J* = Q_tot at the end of a long cold solve; t_tol is the wall-clock
time from the start (warm: including the evaluation at zero and the network inference)
to the first evaluation with Q_tot <= (1 + 1e-4) J*, same solver and settings.

Cold solves for training targets and for J* are spread over worker processes (each with
its own plans on the one GPU); the timed comparison runs in the main process, one field
at a time.

    python -m paper_2609_17636_amd.warmstart --train 1024 --heldout 32 --epochs 40
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

PEAK_K = 50.0
HELDOUT_BASE = 100_000
LAYOUT_SEED = 5001
TOL = 1e-4


# ----------------------------------------------------------------------------- problem
class Mosaic:
    """The warm-start mosaic on the GPU: a float plan for solving and an FP64 plan that
    generates the data."""

    def __init__(self, layout_seed: int = LAYOUT_SEED):
        import synth
        from . import Plan

        p = synth.config_c5_geometry(layout_seed)
        p.vis = np.zeros(p.n_vis, dtype=np.complex64)
        self.problem = p
        self.plan = Plan.from_problem(p)
        self.plan.set_problem_data(p)
        self.plan64 = Plan.from_problem(p, precision="f64")
        self.plan64.set_problem_data(p)
        self.offsets = [int(v) for v in p.vis_offsets]
        self.n = p.n_sky

    @staticmethod
    def field(seed: int) -> np.ndarray:
        import synth

        return synth.lognormal_field(synth.grf_k3(np.random.default_rng(seed), 256), PEAK_K)[None]

    def simulate(self, seed: int) -> np.ndarray:
        """Load the data of field `seed` into the float plan; returns the true sky."""
        import torch

        x = self.field(seed)
        mv = self.plan64.forward(torch.tensor(x, dtype=torch.float64, device="cuda"))
        gen = torch.Generator(device="cuda")
        gen.manual_seed(int(seed))
        noise = torch.randn(mv.shape, generator=gen, device="cuda", dtype=torch.float64)
        w = torch.empty(mv.shape[0], dtype=torch.float64, device="cuda")
        for b in range(len(self.offsets) - 1):
            s = slice(self.offsets[b], self.offsets[b + 1])
            if s.stop == s.start:
                continue
            sig = 0.01 * torch.sqrt((mv[s] ** 2).sum(dim=1)).max()
            mv[s] += sig * noise[s]
            w[s] = 1.0 / (sig * sig)
        self.plan.set_vis(mv.to(torch.float32), w.to(torch.float32))
        return x

    def dirty(self):
        """Normalised dirty mosaic d = -grad Q_tot(0) / max|d| (cuda [1][n][n])."""
        import torch

        _, g = self.plan.objective_grad(torch.zeros((1, self.n, self.n), dtype=torch.float32, device="cuda"))
        d = -g
        return d / d.abs().max().clamp_min(1e-30)


# ----------------------------------------------------------------------------- workers
_MOSAIC = None


def _init_worker():
    global _MOSAIC
    _MOSAIC = Mosaic()


def _cold_one(args):
    """Cold solve of one field: its dirty mosaic, the solution / 50 K (float32) and the
    solve's figures."""
    from .solver import solve

    seed, maxiter = args
    m = _MOSAIC
    m.simulate(seed)
    d = m.dirty().cpu().numpy()[0].astype(np.float32)
    r = solve(m.plan, maxiter=maxiter)
    return {"seed": int(seed), "d": d, "x": (r.x[0] / PEAK_K).astype(np.float32), "fun": float(r.fun),
            "nit": int(r.nit), "nfev": int(r.nfev), "seconds": float(r.seconds), "message": r.message}


def cold_solves(seeds, maxiter, pool=None, log=None, every=32):
    """Cold solves of `seeds`, in the pool's worker processes when given (each holds its
    own plans), else in this process."""
    tasks = [(int(s), int(maxiter)) for s in seeds]
    if pool is None:
        if _MOSAIC is None:
            _init_worker()
        it = map(_cold_one, tasks)
    else:
        it = pool.imap_unordered(_cold_one, tasks, chunksize=1)
    out = []
    for r in it:
        out.append(r)
        if log and len(out) % every == 0:
            log(f"  {len(out)}/{len(tasks)} solves")
    return sorted(out, key=lambda r: r["seed"])


# ----------------------------------------------------------------------------- training
def train(net, D, X, epochs, batch, lr, seed=0, log=None):
    """Adam on the MSE between net(d) and x*/50 K; D, X cuda [n][H][W]."""
    import torch

    rng = np.random.default_rng(seed)
    n = D.shape[0]
    hist = []
    for ep in range(epochs):
        order = rng.permutation(n)
        tot, cnt = 0.0, 0
        for i in range(0, n - batch + 1, batch):
            idx = torch.as_tensor(order[i:i + batch], device=D.device)
            loss = net.train_step(D.index_select(0, idx), X.index_select(0, idx), lr)
            tot += loss
            cnt += 1
        hist.append(tot / max(cnt, 1))
        if log:
            log(f"epoch {ep + 1}/{epochs} train mse {hist[-1]:.5f}")
    return hist


def predict(net, d):
    """x0 = 50 K * max(net(d), 0) for one dirty mosaic d (cuda [1][n][n])."""
    import torch

    y = net.forward(d.contiguous())
    return torch.clamp(y, min=0.0) * PEAK_K


# ----------------------------------------------------------------------------- timing
def time_to_tolerance(m: Mosaic, net, seed: int, j_star: float, maxiter: int = 5000, x_mean=None):
    """Cold and warm time-to-tolerance on field `seed` (data loaded here, untimed).  With
    `x_mean` (sky, K) a third solve starts from that fixed image: the no-learning baseline."""
    import torch

    from .solver import solve

    target = (1.0 + TOL) * j_star
    m.simulate(seed)
    torch.cuda.synchronize()
    cold = solve(m.plan, maxiter=maxiter, target=target)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    d = m.dirty()
    x0 = predict(net, d)
    torch.cuda.synchronize()
    t_pred = time.perf_counter() - t0
    warm = solve(m.plan, x0=x0.cpu().numpy(), maxiter=maxiter, target=target, t_start=t0)
    q0_warm = warm.history[0][1] if warm.history else float("nan")
    extra = {}
    if x_mean is not None:
        mean = solve(m.plan, x0=np.asarray(x_mean), maxiter=maxiter, target=target)
        extra = {"mean_s": mean.seconds if mean.reached_target else float("inf"), "mean_nfev": mean.nfev}
    return {"seed": seed, "j_star": j_star, **extra,
            "cold_s": cold.seconds if cold.reached_target else float("inf"), "cold_nfev": cold.nfev,
            "warm_s": warm.seconds if warm.reached_target else float("inf"), "warm_nfev": warm.nfev,
            "warm_overhead_s": t_pred, "q_warm_start": q0_warm,
            "cold_reached": cold.reached_target, "warm_reached": warm.reached_target}


def summarise(rows):
    c = np.array([r["cold_s"] for r in rows])
    w = np.array([r["warm_s"] for r in rows])
    ok = np.isfinite(c) & np.isfinite(w)
    q = lambda a, p: float(np.percentile(a[np.isfinite(a)], p)) if np.isfinite(a).any() else float("nan")
    return {"fields": len(rows), "both_reached": int(ok.sum()),
            "cold_s_median": q(c, 50), "cold_s_iqr": [q(c, 25), q(c, 75)],
            "warm_s_median": q(w, 50), "warm_s_iqr": [q(w, 25), q(w, 75)],
            "speedup_median": float(np.median(c[ok] / w[ok])) if ok.any() else float("nan"),
            "warm_wins_fraction": float(np.mean(w < c)),
            "cold_nfev_median": float(np.median([r["cold_nfev"] for r in rows])),
            "warm_nfev_median": float(np.median([r["warm_nfev"] for r in rows])),
            "warm_overhead_s_median": float(np.median([r["warm_overhead_s"] for r in rows])),
            "mean_image_s_median": q(np.array([r.get("mean_s", np.nan) for r in rows]), 50),
            "mean_image_nfev_median": float(np.median([r.get("mean_nfev", np.nan) for r in rows]))}


def unet_flops(levels=4, base=32, height=256, width=256, in_ch=4) -> float:
    """Multiply-add FLOPs (2 per MAC) of the 3x3 convolutions of one forward pass of one
    image; a training step costs about three times that (forward, input and weight
    gradients)."""
    ch = [base << l for l in range(levels)]
    f, prev = 0.0, in_ch
    for l in range(levels):
        px = (height >> l) * (width >> l)
        f += 2.0 * px * 9 * (prev * ch[l] + ch[l] * ch[l])
        prev = ch[l]
    for l in range(levels - 2, -1, -1):
        px = (height >> l) * (width >> l)
        f += 2.0 * px * 9 * ((ch[l + 1] + ch[l]) * ch[l] + ch[l] * ch[l])
    return f


# ----------------------------------------------------------------------------- driver
def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--train", type=int, default=1024, help="training fields (seeds 0..N-1)")
    ap.add_argument("--heldout", type=int, default=32, help="held-out fields (seeds 100000..)")
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--solve-iters", type=int, default=800, help="L-BFGS-B iterations of a training target")
    ap.add_argument("--jstar-iters", type=int, default=5000, help="iteration cap of the J* solve")
    ap.add_argument("--workers", type=int, default=12)
    ap.add_argument("--out", default="", help="write the JSON report here too")
    a = ap.parse_args(argv)

    def log(msg):
        print(f"# [{time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)

    import multiprocessing as mp

    pool = None
    if a.workers > 1:
        # host side of each worker's solver single-threaded: the workers share the host cores
        for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
            os.environ[k] = "1"
        pool = mp.get_context("spawn").Pool(a.workers, initializer=_init_worker)
    t0 = time.perf_counter()
    train_seeds = list(range(a.train))
    held = [HELDOUT_BASE + i for i in range(a.heldout)]
    log(f"cold solves: {a.train} training fields x {a.solve_iters} iterations, {a.heldout} held-out to convergence")
    tr = cold_solves(train_seeds, a.solve_iters, pool, log)
    log(f"training targets done ({time.perf_counter() - t0:.0f} s; median {np.median([r['seconds'] for r in tr]):.2f} s, "
        f"{np.median([r['nfev'] for r in tr]):.0f} evaluations per solve)")
    hv = cold_solves(held, a.jstar_iters, pool, log, every=8)
    log(f"J* solves done ({time.perf_counter() - t0:.0f} s; median {np.median([r['nit'] for r in hv]):.0f} iterations)")
    if pool is not None:
        pool.close()
        pool.join()

    import torch

    from .unet import UNet

    D = torch.tensor(np.stack([r["d"] for r in tr]), device="cuda")
    X = torch.tensor(np.stack([r["x"] for r in tr]), device="cuda")
    Dv = torch.tensor(np.stack([r["d"] for r in hv]), device="cuda")
    Xv = torch.tensor(np.stack([r["x"] for r in hv]), device="cuda")
    net = UNet(levels=4, base=32, max_batch=a.batch, height=256, width=256, seed=0)
    t1 = time.perf_counter()
    hist = train(net, D, X, a.epochs, a.batch, a.lr, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    val = []
    for i in range(0, Dv.shape[0], a.batch):
        y = net.forward(Dv[i:i + a.batch])
        val.append(float(((y - Xv[i:i + a.batch]) ** 2).mean()) * y.shape[0])
    val_mse = sum(val) / max(Dv.shape[0], 1)
    base_mse = float(((Xv - X.mean(dim=0, keepdim=True)) ** 2).mean())
    log(f"trained {a.epochs} epochs in {t_train:.0f} s; held-out mse {val_mse:.5f} (mean-image baseline {base_mse:.5f})")

    steps = a.epochs * (D.shape[0] // a.batch)
    step_ms = 1e3 * t_train / max(steps, 1)
    tflops = 3 * unet_flops() * a.batch / (step_ms * 1e-3) / 1e12 if steps else float("nan")
    log(f"training step {step_ms:.2f} ms (batch {a.batch}), ~{tflops:.1f} TFLOP/s on the convolutions")
    x_mean = (X.mean(dim=0, keepdim=True) * PEAK_K).cpu().numpy()
    m = _MOSAIC if _MOSAIC is not None else Mosaic()
    rows = []
    for r in hv:
        rows.append(time_to_tolerance(m, net, r["seed"], r["fun"], a.jstar_iters, x_mean=x_mean))
        log(f"seed {r['seed']}: cold {rows[-1]['cold_s']:.2f} s ({rows[-1]['cold_nfev']} evals), "
            f"warm {rows[-1]['warm_s']:.2f} s ({rows[-1]['warm_nfev']} evals), "
            f"mean image {rows[-1]['mean_s']:.2f} s ({rows[-1]['mean_nfev']} evals)")
    report = {"workload": "warm-start mosaic: 256^2 sky at 30 arcsec, 3x3 hex of 20' beams, 1.8 M visibilities, "
                          "lambda_r 1e-2",
              "train_fields": a.train, "heldout_fields": a.heldout, "target_iterations": a.solve_iters,
              "epochs": a.epochs, "batch": a.batch, "lr": a.lr, "train_seconds": t_train,
              "train_step_ms": step_ms, "train_conv_tflops": tflops,
              "train_mse_last": hist[-1] if hist else None, "heldout_mse": val_mse,
              "heldout_mse_mean_image": base_mse, "tolerance": TOL,
              "summary": summarise(rows), "fields": rows,
              "total_seconds": time.perf_counter() - t0}
    line = json.dumps(report)
    print(line, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(line + "\n")
    return report


if __name__ == "__main__":
    main()
