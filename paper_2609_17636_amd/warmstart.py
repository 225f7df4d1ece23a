"""Learned warm start of the Classic3D solve, and its time-to-tolerance measurement.

The paper solves every field from the null prior x0 = 0 (Sect. 3.4).  Here a 4-level
U-Net (include/ivx_unet.h) maps the normalised dirty mosaic d = -grad Q_tot(0) / max|d|
to a first guess, trained on converged cold-start solutions of the same objective, and the
solve starts from x0 = max(50 K * net(d), 0.3 x_mean) instead, x_mean the mean training
solution.  The floor keeps the start off the bound x >= 0: about a quarter of the network's
raw output is <= 0, and clamped there those pixels make the solver walk Cauchy breakpoints
on every iteration (its most expensive step).  The factor 0.3 was chosen from
{0, 0.02, 0.1, 0.3} on validation fields (training seeds), never on the held-out fields; the
plain clamp max(50 K * net(d), 0) is measured beside it.

Workload (warm-start mosaic): 256^2 sky at 30", 3 x 3 hexagonal mosaic of 20' Gaussian
beams at 40 px pitch, 128^2 sub-images, 200,000 visibilities per pointing (1.8 M),
lambda_r = 1e-2, no single-dish term.  Each field seed gives a k^-3 log-normal sky
(0-50 K); its visibilities are the FP64 HIP forward of that sky plus complex Gaussian noise
of 1% of the peak model amplitude per pointing (natural weights), the noise drawn from a
device generator seeded with the field seed.

Time-to-tolerance: J* = Q_tot at the end of a long cold solve; t_tol is the wall-clock
time from the start (warm: including the evaluation at zero and the network inference)
to the first evaluation with Q_tot <= (1 + 1e-4) J*.  Every solve, cold or warm, is the
device L-BFGS-B loop (include/ivx_lbfgsb.h) with the same settings.

    python -m paper_2609_17636_amd.warmstart --train 512 --heldout 32 --epochs 40

The cold solves that produce training targets and J* run in several host threads, each
with its own plan, device solver and stream (the solver waits on a few scalars per
iteration, so one solve leaves the GPU mostly idle); time-to-tolerance runs one solve at a
time.  `--phase train --save DIR` stops after training and writes the network, the mean
training solution and the J* values; `--phase measure --load DIR` times them.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

PEAK_K = 50.0
HELDOUT_BASE = 100_000
LAYOUT_SEED = 5001
TOL = 1e-4
WARM_FLOOR = 0.3  # floor of the learned start, in units of the mean training solution


# ----------------------------------------------------------------------------- problem
class Mosaic:
    """The warm-start mosaic on the GPU: a float plan and its device solver for solving,
    and an FP64 plan that generates the data."""

    def __init__(self, layout_seed: int = LAYOUT_SEED, autotune_ms: float = 500.0, blocking=None):
        import torch

        import synth
        from . import Plan
        from .solver import DeviceSolver

        p = synth.config_c5_geometry(layout_seed)
        p.vis = np.zeros(p.n_vis, dtype=np.complex64)
        self.problem = p
        self.plan = Plan.from_problem(p)
        self.plan.set_problem_data(p)
        self.plan64 = Plan.from_problem(p, precision="f64")
        self.plan64.set_problem_data(p)
        self.offsets = [int(v) for v in p.vis_offsets]
        self.n = p.n_sky
        self.simulate(0)
        if blocking is not None:
            self.plan.set_blocking(*blocking)
        elif autotune_ms > 0:
            self.plan.autotune(autotune_ms)
        self.solver = DeviceSolver(self.plan)
        self.zero = torch.zeros((1, self.n, self.n), dtype=torch.float32, device="cuda")
        self.grad0 = torch.empty_like(self.zero)

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
        self.plan.objective_grad(self.zero, grad=self.grad0)
        d = -self.grad0
        return d / d.abs().max().clamp_min(1e-30)

    def solve(self, x0=None, **kw):
        return self.solver.solve(x0=x0, **kw)


def cold_solves(m: Mosaic, seeds, maxiter, log=None, every=32):
    """Cold solves of `seeds`: dirty mosaics D, solutions / 50 K X (cuda [n][N][N]) and
    per-field figures."""
    import torch

    D = torch.empty((len(seeds), m.n, m.n), dtype=torch.float32, device="cuda")
    X = torch.empty_like(D)
    info = []
    for i, s in enumerate(seeds):
        m.simulate(s)
        D[i] = m.dirty()[0]
        r = m.solve(maxiter=maxiter)
        X[i] = r.x[0] / PEAK_K
        info.append({"seed": int(s), "fun": r.fun, "nit": r.nit, "nfev": r.nfev, "seconds": r.seconds,
                     "message": r.message})
        if log and (i + 1) % every == 0:
            log(f"  {i + 1}/{len(seeds)} solves")
    return D, X, info


def blocking_of(m: Mosaic):
    i = m.plan.info()
    return (i["tile"], i["waves_per_block"], i["chunk"], i["lanes"], i["vpi"])


def cold_solves_parallel(mosaics, seeds, maxiter, log=None, every=64):
    """cold_solves over several mosaics (one host thread and one stream each); results in
    seed order, identical to a sequential run (each solve only depends on its seed)."""
    import threading

    import torch

    n = mosaics[0].n
    D = torch.empty((len(seeds), n, n), dtype=torch.float32, device="cuda")
    X = torch.empty_like(D)
    torch.cuda.synchronize()
    info = [None] * len(seeds)
    streams = [torch.cuda.Stream() for _ in mosaics]
    lock = threading.Lock()
    state = {"done": 0, "errors": []}

    def work(w):
        m = mosaics[w]
        try:
            with torch.cuda.stream(streams[w]):
                for i in range(w, len(seeds), len(mosaics)):
                    s = seeds[i]
                    m.simulate(s)
                    D[i] = m.dirty()[0]
                    r = m.solve(maxiter=maxiter)
                    X[i] = r.x[0] / PEAK_K
                    info[i] = {"seed": int(s), "fun": r.fun, "nit": r.nit, "nfev": r.nfev, "seconds": r.seconds,
                               "message": r.message}
                    with lock:
                        state["done"] += 1
                        k = state["done"]
                    if log and k % every == 0:
                        log(f"  {k}/{len(seeds)} solves")
            streams[w].synchronize()
        except BaseException as e:  # surfaced after the join
            state["errors"].append(e)

    threads = [threading.Thread(target=work, args=(w,)) for w in range(len(mosaics))]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize()
    if state["errors"]:
        raise state["errors"][0]
    return D, X, info


# ----------------------------------------------------------------------------- training
def mse(net, D, X, batch):
    """Mean squared error of net(D) against X (cuda [n][H][W])."""
    tot = 0.0
    for i in range(0, D.shape[0], batch):
        y = net.forward(D[i:i + batch])
        tot += float(((y - X[i:i + batch]) ** 2).sum())
    return tot / max(X.numel(), 1)


def train(net, D, X, epochs, batch, lr, seed=0, log=None, Dv=None, Xv=None, val_every=5, lr_final=None):
    """Adam on the MSE between net(d) and x*/50 K; D, X cuda [n][H][W].  With lr_final the
    step size follows a cosine from lr to lr_final over the epochs.  With a validation set
    (Dv, Xv: fields not trained on) the parameters of the epoch with the lowest validation
    MSE (checked every val_every epochs) are restored at the end.  Returns (per-epoch
    training MSE, (best validation MSE, its epoch) or None)."""
    import math

    import torch

    rng = np.random.default_rng(seed)
    n = D.shape[0]
    hist = []
    best = (float("inf"), None, 0)
    for ep in range(epochs):
        step_lr = lr if lr_final is None else lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * ep / epochs))
        order = rng.permutation(n)
        tot, cnt = 0.0, 0
        for i in range(0, n - batch + 1, batch):
            idx = torch.as_tensor(order[i:i + batch], device=D.device)
            tot += net.train_step(D.index_select(0, idx), X.index_select(0, idx), step_lr)
            cnt += 1
        hist.append(tot / max(cnt, 1))
        msg = f"epoch {ep + 1}/{epochs} train mse {hist[-1]:.6f} lr {step_lr:.2e}"
        if Dv is not None and ((ep + 1) % val_every == 0 or ep + 1 == epochs):
            v = mse(net, Dv, Xv, batch)
            msg += f" validation mse {v:.6f}"
            if v < best[0]:
                best = (v, net.get_params().copy(), ep + 1)
        if log:
            log(msg)
    if best[1] is not None:
        net.set_params(best[1])
        return hist, (best[0], best[2])
    return hist, None


def predict(net, d, floor=None):
    """Learned start for one dirty mosaic d (cuda [1][n][n]): 50 K * net(d), raised to
    `floor` (a cuda image, e.g. WARM_FLOOR * the mean training solution) or, with no floor,
    clamped at 0."""
    import torch

    x = net.forward(d.contiguous()) * PEAK_K
    return torch.clamp(x, min=0.0) if floor is None else torch.maximum(x, floor)


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


# ----------------------------------------------------------------------------- timing
def time_to_tolerance(m: Mosaic, net, seed: int, j_star: float, maxiter: int = 15000, x_mean=None, order: int = 0):
    """Cold and warm time-to-tolerance on field `seed` (data loaded here, untimed).  With
    `x_mean` (sky, K, the mean training solution) the learned start is floored at
    WARM_FLOOR * x_mean, and two more solves run: from the plain clamp max(50 K net(d), 0)
    ("clamp", the ablation of the floor) and from x_mean itself ("mean", the no-learning
    baseline).  `order` rotates which start is solved first, so that no start always runs on
    a cold cache or right after another solve."""
    import torch

    target = (1.0 + TOL) * j_star
    m.simulate(seed)
    torch.cuda.synchronize()
    res = {}

    def run_cold():
        res["cold"] = m.solve(maxiter=maxiter, target=target)
        torch.cuda.synchronize()

    def run_warm():
        t0 = time.perf_counter()
        d = m.dirty()
        x0 = predict(net, d, None if x_mean is None else WARM_FLOOR * x_mean)
        torch.cuda.synchronize()
        res["t_pred"] = time.perf_counter() - t0
        res["warm"] = m.solve(x0=x0, maxiter=maxiter, target=target, t_start=t0)
        torch.cuda.synchronize()

    def run_clamp():
        t0 = time.perf_counter()
        x0 = predict(net, m.dirty())
        torch.cuda.synchronize()
        res["clamp"] = m.solve(x0=x0, maxiter=maxiter, target=target, t_start=t0)
        torch.cuda.synchronize()

    def run_mean():
        res["mean"] = m.solve(x0=x_mean, maxiter=maxiter, target=target)
        torch.cuda.synchronize()

    steps = [run_cold, run_warm] + ([run_mean, run_clamp] if x_mean is not None else [])
    k = order % len(steps)
    for f in steps[k:] + steps[:k]:
        f()
    cold, warm, t_pred = res["cold"], res["warm"], res["t_pred"]
    row = {"seed": seed, "j_star": j_star, "order": k,
           "cold_s": cold.seconds if cold.reached_target else float("inf"), "cold_nfev": cold.nfev,
           "warm_s": warm.seconds if warm.reached_target else float("inf"), "warm_nfev": warm.nfev,
           "warm_overhead_s": t_pred, "q_warm_start": warm.history[0][1] if warm.history else float("nan"),
           "q_cold_start": cold.history[0][1] if cold.history else float("nan")}
    names = ("cold", "warm") + (("mean", "clamp") if x_mean is not None else ())
    for name in names[2:]:
        r = res[name]
        row.update({f"{name}_s": r.seconds if r.reached_target else float("inf"), f"{name}_nfev": r.nfev})
    for name in names:
        r = res[name]
        row[f"{name}_ms_per_eval"] = 1e3 * r.seconds / max(r.nfev, 1) if np.isfinite(r.seconds) else float("nan")
        row[f"{name}_walks"] = r.n_walks
    return row


def summarise(rows):
    c = np.array([r["cold_s"] for r in rows])
    w = np.array([r["warm_s"] for r in rows])
    ok = np.isfinite(c) & np.isfinite(w)

    def q(a, p):
        a = np.asarray(a, dtype=float)
        a = a[np.isfinite(a)]
        return float(np.percentile(a, p)) if a.size else float("nan")

    return {"fields": len(rows), "both_reached": int(ok.sum()),
            "cold_s_median": q(c, 50), "cold_s_iqr": [q(c, 25), q(c, 75)],
            "warm_s_median": q(w, 50), "warm_s_iqr": [q(w, 25), q(w, 75)],
            "speedup_median": float(np.median(c[ok] / w[ok])) if ok.any() else float("nan"),
            "warm_wins_fraction": float(np.mean(w < c)),
            "cold_nfev_median": float(np.median([r["cold_nfev"] for r in rows])),
            "warm_nfev_median": float(np.median([r["warm_nfev"] for r in rows])),
            "warm_overhead_s_median": float(np.median([r["warm_overhead_s"] for r in rows])),
            "mean_image_s_median": q([r.get("mean_s", np.nan) for r in rows], 50),
            "mean_image_s_iqr": [q([r.get("mean_s", np.nan) for r in rows], p) for p in (25, 75)],
            "mean_image_nfev_median": q([r.get("mean_nfev", np.nan) for r in rows], 50),
            "clamp_s_median": q([r.get("clamp_s", np.nan) for r in rows], 50),
            "clamp_s_iqr": [q([r.get("clamp_s", np.nan) for r in rows], p) for p in (25, 75)],
            "clamp_nfev_median": q([r.get("clamp_nfev", np.nan) for r in rows], 50),
            "warm_vs_mean_wins_fraction": float(np.mean([r["warm_s"] < r.get("mean_s", np.inf) for r in rows])),
            "warm_vs_mean_fewer_evals_fraction": float(np.mean([r["warm_nfev"] < r.get("mean_nfev", np.inf)
                                                                for r in rows])),
            "speedup_vs_mean_median": q([r.get("mean_s", np.nan) / r["warm_s"] for r in rows], 50),
            "ms_per_eval_median": {k: q([r.get(f"{k}_ms_per_eval", np.nan) for r in rows], 50)
                                   for k in ("cold", "warm", "mean", "clamp")},
            "walks_median": {k: q([r.get(f"{k}_walks", np.nan) for r in rows], 50)
                             for k in ("cold", "warm", "mean", "clamp")}}


def select_floor(m: Mosaic, net, x_mean, seeds, floors=(0.0, 0.02, 0.1, 0.3), maxiter: int = 15000, log=None):
    """Time-to-tolerance of the learned start max(50 K net(d), f x_mean) for each candidate
    floor f (f = 0: the plain clamp at 0), beside the cold and the mean-image starts, on
    `seeds` (validation fields: J* from a cold solve here).  Returns per-start medians."""
    import torch

    rows = []
    for s in seeds:
        m.simulate(s)
        target = (1.0 + TOL) * m.solve(maxiter=maxiter).fun
        raw = net.forward(m.dirty().contiguous()) * PEAK_K
        starts = {"cold": None, "mean": x_mean}
        for f in floors:
            starts[f"floor {f:g}"] = torch.clamp(raw, min=0.0) if f == 0 else torch.maximum(raw, f * x_mean)
        row = {"seed": s, "raw_le_0_fraction": float((raw <= 0).float().mean())}
        for k, x0 in starts.items():
            r = m.solve(x0=x0, maxiter=maxiter, target=target)
            torch.cuda.synchronize()
            row[k] = {"s": r.seconds if r.reached_target else float("inf"), "nfev": r.nfev, "nit": r.nit,
                      "walks": r.n_walks}
        rows.append(row)
        if log:
            log(f"seed {s}: " + ", ".join(f"{k} {row[k]['s']:.3f} s" for k in starts))
    keys = [k for k in rows[0] if isinstance(rows[0][k], dict)]
    med = {k: {q: float(np.median([r[k][q] for r in rows])) for q in ("s", "nfev", "nit", "walks")} for k in keys}
    for k in keys:
        med[k]["ms_per_eval"] = float(np.median([1e3 * r[k]["s"] / r[k]["nfev"] for r in rows]))
    return {"seeds": [int(s) for s in seeds], "median": med,
            "raw_le_0_fraction_median": float(np.median([r["raw_le_0_fraction"] for r in rows])), "fields": rows}


# ----------------------------------------------------------------------------- command line
def solve_timing(iters: int = 200, repeats: int = 5) -> dict:
    """Cold device solve of the first held-out field for `iters` iterations (after a
    30-iteration warm-up solve), repeated: wall-clock per evaluation (median and minimum over
    the repeats; every repeat runs the same iterates), and how many iterations walked the
    Cauchy breakpoints."""
    import torch

    m = Mosaic()
    m.simulate(HELDOUT_BASE)
    m.solve(maxiter=30)
    torch.cuda.synchronize()
    runs = []
    for _ in range(max(repeats, 1)):
        r = m.solve(maxiter=iters)
        torch.cuda.synchronize()
        runs.append(1e3 * r.seconds / max(r.nfev, 1))
    return {"workload": "warm-start mosaic, cold solve of field 100000", "iterations": r.nit, "evaluations": r.nfev,
            "walks": r.n_walks, "seconds": r.seconds, "repeats": len(runs), "ms_per_eval": float(np.median(runs)),
            "ms_per_eval_min": min(runs)}


def train_throughput(batch: int = 16, steps: int = 50, warmup: int = 5) -> dict:
    """Training steps of the warm-start network (forward, backward, Adam) on a random batch of
    256^2 fields: milliseconds per step and the convolutions' rate against the dense bf16 matrix
    peak of MI355X (2.5 PFLOP/s)."""
    import torch

    from .unet import UNet

    net = UNet(levels=4, base=32, max_batch=batch, height=256, width=256, seed=0)
    g = torch.Generator(device="cuda").manual_seed(0)
    d = torch.rand((batch, 256, 256), generator=g, device="cuda")
    x = torch.rand((batch, 256, 256), generator=g, device="cuda")
    for _ in range(warmup):
        net.train_step(d, x, 1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        net.train_step(d, x, 1e-4)
    torch.cuda.synchronize()
    step_ms = 1e3 * (time.perf_counter() - t0) / steps
    tflops = 3 * unet_flops() * batch / (step_ms * 1e-3) / 1e12
    return {"batch": batch, "steps": steps, "train_step_ms": step_ms, "conv_tflops": tflops,
            "peak_tflops": 2500.0, "frac": tflops / 2500.0}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--train", type=int, default=512, help="training fields (seeds 0..N-1)")
    ap.add_argument("--heldout", type=int, default=32, help="held-out fields (seeds 100000..)")
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--solve-iters", type=int, default=15000,
                    help="iteration cap of a training target's cold solve (15000: run to the stopping rule)")
    ap.add_argument("--jstar-iters", type=int, default=15000, help="iteration cap of the J* solve")
    ap.add_argument("--out", default="", help="write the JSON report here too")
    ap.add_argument("--workers", type=int, default=8, help="host threads (plans) for the untimed cold solves")
    ap.add_argument("--val", type=int, default=0,
                    help="training fields held back to select the epoch (validation, not the held-out test set)")
    ap.add_argument("--lr-final", type=float, default=None, help="cosine step-size schedule from --lr to this")
    ap.add_argument("--phase", default="all",
                    choices=("all", "train", "measure", "throughput", "solve", "select-floor"),
                    help="throughput: time --steps training steps of the network on random fields only; "
                         "solve: time one cold device solve of --solve-iters iterations (first held-out field); "
                         "select-floor: time the learned start under each candidate floor on --val-fields "
                         "validation fields (the last training seeds) with the network of --load")
    ap.add_argument("--val-fields", type=int, default=24, help="--phase select-floor: validation fields")
    ap.add_argument("--steps", type=int, default=50, help="--phase throughput: timed training steps")
    ap.add_argument("--save", default="", help="--phase train: directory for the network, mean image and J*")
    ap.add_argument("--load", default="", help="--phase measure: directory written by --phase train")
    a = ap.parse_args(argv)

    def log(msg):
        print(f"# [{time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)

    import torch

    from .unet import UNet

    import os

    if a.phase == "throughput":
        print(json.dumps(train_throughput(a.batch, a.steps)), flush=True)
        return
    if a.phase == "solve":
        print(json.dumps(solve_timing(a.solve_iters)), flush=True)
        return
    t0 = time.perf_counter()
    m = Mosaic()
    log(f"mosaic ready ({time.perf_counter() - t0:.1f} s): {m.plan.info()}")
    net = UNet(levels=4, base=32, max_batch=a.batch, height=256, width=256, seed=0)
    if a.phase == "select-floor":
        net.set_params(np.load(os.path.join(a.load, "unet_params.npy")))
        x_mean = torch.tensor(np.load(os.path.join(a.load, "x_mean.npy")), device="cuda")
        with open(os.path.join(a.load, "warmstart_train.json")) as f:
            n_train = json.load(f)["report"]["train_fields"]
        seeds = list(range(n_train - a.val_fields, n_train))
        out = select_floor(m, net, x_mean, seeds, log=log)
        print(json.dumps(out), flush=True)
        if a.out:
            with open(a.out, "w") as f:
                json.dump(out, f)
        return out
    if a.phase == "measure":
        with open(os.path.join(a.load, "warmstart_train.json")) as f:
            saved = json.load(f)
        net.set_params(np.load(os.path.join(a.load, "unet_params.npy")))
        x_mean = torch.tensor(np.load(os.path.join(a.load, "x_mean.npy")), device="cuda")
        hv = saved["jstar"]
        report = dict(saved["report"])
        log(f"loaded network, mean image and {len(hv)} J* values from {a.load}")
        return _measure(a, m, net, hv, x_mean, report, t0, log)
    extra = [Mosaic(autotune_ms=0.0, blocking=blocking_of(m)) for _ in range(max(a.workers, 1) - 1)]
    log(f"{len(extra) + 1} solver threads ready ({time.perf_counter() - t0:.1f} s)")
    log(f"cold solves: {a.train} training fields x {a.solve_iters} iterations")
    t_s = time.perf_counter()
    D, X, tr = cold_solves_parallel([m] + extra, list(range(a.train)), a.solve_iters, log)
    log(f"training targets done ({time.perf_counter() - t_s:.0f} s; median {np.median([r['seconds'] for r in tr]):.3f} s, "
        f"{np.median([r['nfev'] for r in tr]):.0f} evaluations per solve, {len(extra) + 1} threads)")
    held = [HELDOUT_BASE + i for i in range(a.heldout)]
    Dv, Xv, hv = cold_solves_parallel([m] + extra, held, a.jstar_iters, log, every=16)
    log(f"J* solves done ({time.perf_counter() - t0:.0f} s; median {np.median([r['nit'] for r in hv]):.0f} iterations, "
        f"{np.median([r['seconds'] for r in hv]):.2f} s, stop {sorted(set(r['message'] for r in hv))})")
    del extra

    torch.cuda.synchronize()
    n_fit = D.shape[0] - a.val
    Dt, Xt = D[:n_fit], X[:n_fit]
    Dval, Xval = (D[n_fit:], X[n_fit:]) if a.val > 0 else (None, None)
    t1 = time.perf_counter()
    hist, best = train(net, Dt, Xt, a.epochs, a.batch, a.lr, log=log, Dv=Dval, Xv=Xval, lr_final=a.lr_final)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    if best is not None:
        log(f"validation-selected epoch {best[1]} (validation mse {best[0]:.6f} on {a.val} fields)")
    steps = a.epochs * (Dt.shape[0] // a.batch)
    step_ms = 1e3 * t_train / max(steps, 1)
    tflops = 3 * unet_flops() * a.batch / (step_ms * 1e-3) / 1e12 if steps else float("nan")
    val = 0.0
    for i in range(0, Dv.shape[0], a.batch):
        y = net.forward(Dv[i:i + a.batch])
        val += float(((y - Xv[i:i + a.batch]) ** 2).sum())
    val_mse = val / max(Xv.numel(), 1)
    base_mse = float(((Xv - Xt.mean(dim=0, keepdim=True)) ** 2).mean())
    log(f"trained {a.epochs} epochs in {t_train:.0f} s ({step_ms:.1f} ms per step of {a.batch}, "
        f"~{tflops:.1f} TFLOP/s on the convolutions); held-out mse {val_mse:.6f} "
        f"(mean-image baseline {base_mse:.6f})")

    x_mean = Xt.mean(dim=0, keepdim=True) * PEAK_K
    report = {"workload": "warm-start mosaic: 256^2 sky at 30 arcsec, 3x3 hex of 20' beams, 1.8 M visibilities, "
                          "lambda_r 1e-2",
              "solver": "device L-BFGS-B (m 10, x >= 0)",
              "train_fields": a.train, "heldout_fields": a.heldout, "target_iterations": a.solve_iters,
              "epochs": a.epochs, "batch": a.batch, "lr": a.lr, "train_seconds": t_train,
              "train_step_ms": step_ms, "train_conv_tflops": tflops,
              "train_mse_last": hist[-1] if hist else None, "heldout_mse": val_mse,
              "validation_fields": a.val, "lr_final": a.lr_final,
              "selected_epoch": best[1] if best else a.epochs, "validation_mse": best[0] if best else None,
              "heldout_mse_mean_image": base_mse, "tolerance": TOL,
              "target_solves": {"seconds_median": float(np.median([r["seconds"] for r in tr])),
                                "nfev_median": float(np.median([r["nfev"] for r in tr])),
                                "threads": a.workers},
              "jstar_solves": {"seconds_median": float(np.median([r["seconds"] for r in hv])),
                               "nit_median": float(np.median([r["nit"] for r in hv]))}}
    if a.phase == "train":
        os.makedirs(a.save, exist_ok=True)
        np.save(os.path.join(a.save, "unet_params.npy"), net.get_params())
        np.save(os.path.join(a.save, "x_mean.npy"), x_mean.cpu().numpy())
        with open(os.path.join(a.save, "warmstart_train.json"), "w") as f:
            json.dump({"jstar": [{"seed": r["seed"], "fun": r["fun"], "nit": r["nit"], "message": r["message"]}
                                 for r in hv], "report": report}, f)
        log(f"saved network, mean image and J* to {a.save} ({time.perf_counter() - t0:.0f} s)")
        return report
    return _measure(a, m, net, hv, x_mean, report, t0, log)


def _measure(a, m, net, hv, x_mean, report, t0, log):
    rows = []
    for i, r in enumerate(hv):
        rows.append(time_to_tolerance(m, net, r["seed"], r["fun"], a.jstar_iters, x_mean=x_mean, order=i))
        w = rows[-1]
        log(f"seed {r['seed']}: cold {w['cold_s']:.3f} s ({w['cold_nfev']} evals), warm {w['warm_s']:.3f} s "
            f"({w['warm_nfev']} evals), mean image {w['mean_s']:.3f} s ({w['mean_nfev']} evals), "
            f"clamped learned {w['clamp_s']:.3f} s ({w['clamp_nfev']} evals)")
    report = dict(report)
    report.update({"summary": summarise(rows), "fields": rows, "total_seconds": time.perf_counter() - t0})
    line = json.dumps(report)
    print(line, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(line + "\n")
    return report


if __name__ == "__main__":
    main()
