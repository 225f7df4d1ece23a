"""Benchmark: Classic3D objective + gradient evaluations on one MI355X.

A step is one full evaluation of Q_tot(x) and its gradient (primary-beam-weighted forward
NUFFT, residual and data term, adjoint NUFFT, reprojection transpose, Laplacian
regulariser) on the single-pointing workload: 512^2 sky at 7 arcsec of a k^-3 log-normal
field, 630 baselines x 1000 samples = 630,000 visibilities, lambda_r = 1e-2.  Inputs are
resident in HBM before the timed region; the timed region is exactly `--steps`
evaluations bracketed by device synchronisations.

Prints one JSON line: value = visibilities per second (forward + adjoint counted once per
visibility), the roofline of the dominant kernel (HIP events around it on the evaluation
stream, during the timed evaluations) and the FP64 oracle timed on a bounded sample on the
host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Gridding blocking (tile, waves per block, chunk, lanes per visibility, visibilities per
# lane group) that the plan autotuner selects for this workload; fixed so that the counter
# measurements committed beside the benchmark describe the kernel configuration it runs.
DEFAULT_BLOCKING = "8,1,256,64,1"
# blocking the autotuner picks on the 36-pointing mosaic; used for the spectral cube, whose
# per-(pointing, channel) blocks have the mosaic's shape
CUBE_BLOCKING = "10,1,512,64,1"
METRIC = "visibilities/s fwd+adjoint NUFFT; time-to-tol cold vs learned warm start"


def grid_algorithmic_bytes(n_live: int, n_fine: int, real_bytes: int = 4, n_items: int = 1) -> float:
    """Algorithmic HBM bytes of the fused degrid/residual/spread stage for one evaluation:
    the visibility stream (coordinates 2x4 B, data 2 reals, weight 1 real) plus, for each of
    the n_items (pointing, channel) blocks, reading the fine-grid half-plane once and writing
    the adjoint half-plane once (G/2 each, G = n_f^2 complex values)."""
    per_vis = 8 + 3 * real_bytes
    G = n_fine * n_fine * 2 * real_bytes
    return n_live * per_vis + n_items * G


def grid_kernel_name(info: dict) -> str:
    """The gridding kernel a blocking runs: the matrix-core variant for lanes = 64."""
    return "k_gridmx" if info.get("lanes") == 64 else "k_grid"


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_grid_traffic_c2.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_2609_17636_amd", "csrc", "ivx_kernels.hip")


def measured_traffic(blocking: str):
    """HBM bytes per launch of the gridding kernel from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary, or None when the kernel source or the blocking changed since it was
    taken."""
    import hashlib

    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    if kv.get("kernel_source_sha256") != sha or "traffic_bytes_per_launch" not in kv:
        return None
    if kv.get("blocking") != blocking:
        return None
    return float(kv["traffic_bytes_per_launch"])


def copy_probe(steps: int):
    """Plain device copy of 1 GiB, `steps` times: the calibration kernel for the FETCH_SIZE /
    WRITE_SIZE counters (each dispatch, the runtime's __amd_rocclr_copyBuffer, reads and writes
    exactly 2^30 bytes; the fill that creates the source is a different kernel)."""
    import torch

    n = (1 << 30) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_per_dispatch": 1 << 30, "steps": steps}), flush=True)


def build_workload(seed=2001):
    import synth

    return synth.config_c2(seed)


def cpu_baseline(p, target_s=12.0):
    """FP64 oracle (direct DFT forward + explicit adjoint + Laplacian) on a bounded sample of
    the same workload: the first M_s visibilities, M_s grown until ~target_s of CPU work."""
    import oracle

    x = p.x_true
    m_s = 1000
    while True:
        q = _subsample(p, m_s)
        t0 = time.perf_counter()
        oracle.objective_grad(q, x)
        dt = time.perf_counter() - t0
        if dt >= target_s or m_s >= p.n_vis:
            break
        m_s = int(min(p.n_vis, max(m_s * 2, m_s * target_s / max(dt, 1e-3) * 1.05)))
    return {"value": m_s / dt, "unit": "vis/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"one FP64 objective+gradient evaluation over the first {m_s} of {p.n_vis} "
                      f"visibilities (512^2 sky, {dt:.1f} s)", "seconds": dt}


def _subsample(p, m):
    import copy

    q = copy.copy(p)
    q.uv = p.uv[:m]
    q.vis = p.vis[:m]
    q.weight = p.weight[:m]
    q.flags = None if p.flags is None else p.flags[:m]
    q.vis_offsets = np.array([0, m], dtype=np.int64)
    return q


def run_mosaic(args):
    """The 36-pointing mosaic: 1024^2 sky at 30", 6 x 6 hex of 1 deg beams, 384^2
    sub-images, 1400-2000 samples x 630 baselines per pointing with 0-30% flags (about 34 M
    live visibilities), 64 x 64 single-dish map, lambda_r = 1e-2, lambda_s = 1.  Data from the
    FP64 HIP forward of the true sky plus 1% noise per pointing.  Prints one JSON line."""
    import torch

    import synth
    from paper_2609_17636_amd import Plan

    dev = torch.device("cuda:0")
    p = synth.config_c3()
    synth.attach_sd_level(p)
    p.vis = np.zeros(p.n_vis, dtype=np.complex64)
    print(f"# workload {p.name}: N={p.n_sky} vis={p.n_vis} live={int((p.flags == 0).sum())}", file=sys.stderr,
          flush=True)
    plan64 = Plan.from_problem(p, precision="f64")
    plan64.set_problem_data(p)
    mv = plan64.forward(torch.tensor(p.x_true, dtype=torch.float64, device=dev)).cpu().numpy()
    del plan64
    synth.attach_data(p, mv[:, 0] + 1j * mv[:, 1])
    plan = Plan.from_problem(p)
    plan.set_problem_data(p)
    plan.autotune(3000.0)
    info = plan.info()
    print(f"# plan {info}", file=sys.stderr, flush=True)
    rng = np.random.default_rng(0)
    x = torch.tensor(rng.uniform(0, 50, size=p.x_true.shape), dtype=torch.float32, device=dev)
    grad = torch.empty_like(x)
    terms = torch.zeros(4, dtype=torch.float64, device=dev)
    for _ in range(args.warmup):
        plan.objective_grad(x, grad=grad, terms=terms)
    torch.cuda.synchronize()
    plan.set_timing(("grid",))
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.objective_grad(x, grad=grad, terms=terms)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stage_ms, n_timed = plan.stage_times()
    plan.set_timing(())
    n_live = info["n_live_vis"]
    grid_ms = stage_ms["grid"] / max(n_timed, 1)
    alg = grid_algorithmic_bytes(n_live, info["n_fine"], n_items=info["n_items"])
    achieved = alg / (grid_ms * 1e-3) / 1e9
    ms = 1e3 * dt / args.steps
    out = {"metric": METRIC, "value": n_live * args.steps / dt, "unit": "vis/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "36-pointing mosaic, 1024^2 sky at 30 arcsec, 384^2 sub-images, "
                                  f"{n_live} live visibilities, single-dish 64x64, lambda_r=1e-2, lambda_s=1",
                      "n_sky": p.n_sky, "n_vis": n_live, "n_fine": info["n_fine"],
                      "kernel_width": info["kernel_width"], "parallelism": "1 GPU",
                      "blocking": {k: info[k] for k in ("tile", "waves_per_block", "chunk", "lanes", "vpi")}},
           "evals_per_s": 1e3 / ms,
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": grid_kernel_name(info),
                        "kernel_ms": grid_ms, "algorithmic_bytes": alg}}
    print(f"# {ms:.4f} ms/eval, grid {grid_ms:.4f} ms/launch, Q_tot={terms[0].item():.6e}", file=sys.stderr,
          flush=True)
    print(json.dumps(out), flush=True)


def run_cube(args):
    """The spectral cube: 128 channels x 36 pointings x 1024^2 sky (30 arcsec), 384^2
    sub-images, one uv track of 1800 samples x 630 baselines per pointing shared by all
    channels (scaled by nu_c / nu_ref), 0-5% flags per (pointing, channel): about 5.1e9
    live visibilities in one plan, every (pointing, channel, tile) work item in one launch
    per stage.  Data: unit-variance noise (the cost does not depend on the values).
    Prints one JSON line."""
    import torch

    import synth
    from paper_2609_17636_amd import Plan

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    p = synth.config_c4(with_field=False)
    synth.attach_sd_level(p)
    print(f"# workload {p.name}: N={p.n_sky} C={p.n_chan} P={p.n_point} vis={p.n_vis} "
          f"({time.perf_counter() - t0:.1f} s to generate)", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    tile, waves, chunk, lanes, vpi = map(int, args.blocking.split(","))
    plan = Plan.from_problem(p, tile=tile)
    plan.set_cube_data(p)
    if args.autotune:
        plan.autotune(3000.0)
    else:
        plan.set_blocking(tile, waves, chunk, lanes, vpi)
    torch.cuda.synchronize()
    info = plan.info()
    print(f"# plan in {time.perf_counter() - t0:.1f} s: {info}", file=sys.stderr, flush=True)
    n_chan, n_sky = p.n_chan, p.n_sky
    del p
    rng = np.random.default_rng(0)
    x = torch.tensor(rng.uniform(0, 50, size=(n_chan, n_sky, n_sky)).astype(np.float32), device=dev)
    grad = torch.empty_like(x)
    terms = torch.zeros(4, dtype=torch.float64, device=dev)
    for _ in range(args.warmup):
        plan.objective_grad(x, grad=grad, terms=terms)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.objective_grad(x, grad=grad, terms=terms)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # per-stage breakdown from separate, event-timed evaluations
    plan.set_timing()
    for _ in range(3):
        plan.objective_grad(x, grad=grad, terms=terms)
    torch.cuda.synchronize()
    stage_ms, n_timed = plan.stage_times()
    plan.set_timing(())
    n_live = info["n_live_vis"]
    grid_ms = stage_ms["grid"] / max(n_timed, 1)
    alg = grid_algorithmic_bytes(n_live, info["n_fine"], n_items=info["n_items"])
    achieved = alg / (grid_ms * 1e-3) / 1e9
    ms = 1e3 * dt / args.steps
    out = {"metric": METRIC, "value": n_live * args.steps / dt, "unit": "vis/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "spectral cube, 128 channels x 36 pointings, 1024^2 sky at 30 arcsec, 384^2 "
                                  f"sub-images, shared uv per pointing, {n_live} live visibilities, "
                                  "single-dish 64x64 per channel, lambda_r=1e-2, lambda_s=1",
                      "n_sky": 1024, "n_vis": n_live, "n_fine": info["n_fine"],
                      "kernel_width": info["kernel_width"], "parallelism": "1 GPU",
                      "device_bytes": info["device_bytes"],
                      "blocking": {k: info[k] for k in ("tile", "waves_per_block", "chunk", "lanes", "vpi")}},
           "evals_per_s": 1e3 / ms,
           "stage_ms": {k: v / max(n_timed, 1) for k, v in stage_ms.items()},
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": grid_kernel_name(info),
                        "kernel_ms": grid_ms, "algorithmic_bytes": alg}}
    print(f"# {ms:.2f} ms/eval, grid {grid_ms:.2f} ms/launch, Q_tot={terms[0].item():.6e}", file=sys.stderr,
          flush=True)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-probe", action="store_true", help="run the counter calibration copy only")
    ap.add_argument("--blocking", default=DEFAULT_BLOCKING,
                    help="tile,waves,chunk,lanes,vpi of the gridding kernel (default: the autotuner's "
                         "choice for this workload, recorded)")
    ap.add_argument("--autotune", action="store_true", help="run the plan autotuner instead of --blocking")
    ap.add_argument("--workload", default="single", choices=("single", "mosaic", "cube"),
                    help="single: the 512^2 single-pointing benchmark (default); mosaic: the 36-pointing "
                         "1024^2 mosaic (separate measurement line, autotuned); cube: the 128-channel "
                         "spectral cube on the mosaic geometry (separate line; --blocking, default "
                         f"{CUBE_BLOCKING})")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe(args.steps)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: the library runs on one "
              f"GPU (sharding channels and pointings across GPUs is described, not implemented)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "mosaic":
        run_mosaic(args)
        return
    if args.workload == "cube":
        if args.blocking == DEFAULT_BLOCKING:
            args.blocking = CUBE_BLOCKING
        run_cube(args)
        return

    import torch

    import synth
    from paper_2609_17636_amd import Plan

    dev = torch.device("cuda:0")
    p = build_workload()
    print(f"# workload {p.name}: N={p.n_sky} vis={p.n_vis}", file=sys.stderr, flush=True)
    plan = Plan.from_problem(p)
    # data: y = model(x_true) + 1% noise, model from the HIP forward (inputs only)
    p.vis = np.zeros(p.n_vis, dtype=np.complex64)
    plan.set_problem_data(p)
    x_true = torch.tensor(p.x_true, dtype=torch.float32, device=dev)
    mv = plan.forward(x_true).double().cpu().numpy()
    synth.attach_data(p, mv[:, 0] + 1j * mv[:, 1])
    plan.set_problem_data(p)
    if args.autotune:
        plan.autotune(2000.0)
    else:
        plan.set_blocking(*[int(v) for v in args.blocking.split(",")])
    info = plan.info()
    tile = info["tile"]
    blocking = ",".join(str(info[k]) for k in ("tile", "waves_per_block", "chunk", "lanes", "vpi"))
    print(f"# plan {info}", file=sys.stderr, flush=True)

    rng = np.random.default_rng(0)
    x = torch.tensor(rng.uniform(0, 50, size=p.x_true.shape), dtype=torch.float32, device=dev)
    grad = torch.empty_like(x)
    terms = torch.zeros(4, dtype=torch.float64, device=dev)
    for _ in range(args.warmup):
        plan.objective_grad(x, grad=grad, terms=terms)
    torch.cuda.synchronize()
    plan.set_timing(("grid",))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.objective_grad(x, grad=grad, terms=terms)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stage_ms, n_timed = plan.stage_times()
    plan.set_timing(())
    ms_step = 1e3 * dt / args.steps
    vis_s = p.n_vis * args.steps / dt
    grid_ms = stage_ms["grid"] / max(n_timed, 1)
    alg = grid_algorithmic_bytes(info["n_live_vis"], info["n_fine"])
    achieved = alg / (grid_ms * 1e-3) / 1e9
    print(f"# {ms_step:.4f} ms/eval, grid {grid_ms:.4f} ms/launch, Q_tot={terms[0].item():.6e}",
          file=sys.stderr, flush=True)

    out = {
        "metric": METRIC, "value": vis_s, "unit": "vis/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "single-pointing 512x512 sky (7 arcsec, k^-3 log-normal 0-50 K), "
                               "630 baselines x 1000 samples = 630,000 visibilities, lambda_r=1e-2",
                   "n_sky": p.n_sky, "n_vis": p.n_vis, "n_fine": info["n_fine"],
                   "kernel_width": info["kernel_width"], "tile": tile, "parallelism": "1 GPU",
                   "blocking": {k: info[k] for k in ("tile", "waves_per_block", "chunk", "lanes", "vpi")}},
        "evals_per_s": 1e3 / ms_step,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(blocking), "kernel": grid_kernel_name(info),
                     "kernel_ms": grid_ms, "algorithmic_bytes": alg},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
