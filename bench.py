"""Benchmark: Classic3D objective + gradient evaluations on one MI355X.

A step is one full evaluation of Q_tot(x) and its gradient: per (pointing, channel) block
the reprojection, primary-beam weighting and forward NUFFT, residual and data term, the
adjoint NUFFT, the reprojection transpose summed over pointings, the Laplacian regulariser
and the single-dish fusion term, reduced to the four FP64 totals.

Default workload: the spectral cube, the largest single-GPU configuration -- 128 channels x
36 pointings on a 1024^2 sky at 30 arcsec, 384^2 sub-images, one uv track of 630 baselines
x 1800 samples per pointing shared by every channel (scaled by nu_c / nu_ref), 0-5% flags
per (pointing, channel): 5.1e9 live visibilities, single-dish 64 x 64 map per channel,
lambda_r = 1e-2, lambda_s = 1.  `--workload single` / `--workload mosaic` time the
512^2 single-pointing problem and the one-channel 36-pointing mosaic instead.

Inputs are resident in HBM before the timed region.  The timed region is exactly `--steps`
evaluations replayed from the plan's captured HIP graph, bracketed by device
synchronisations, with nothing else on the stream.  A second pass of `--steps`
evaluations launched one by one, with HIP events on the evaluation stream around every
launch of the gridding kernel, gives that kernel's average duration for the roofline; a
third, short pass gives the per-stage breakdown.

Prints one JSON line: value = visibilities per second (forward and adjoint counted once per
visibility), the roofline of the dominant kernel and the FP64 oracle timed on a bounded
sample on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Gridding blockings (tile, waves per block, chunk, lanes per visibility, visibilities per lane
# group) that the plan autotuner selects for each workload; fixed so that the counter
# measurements committed beside the benchmark describe the kernel configuration it runs.
SINGLE_BLOCKING = "8,1,256,64,1"
MOSAIC_W_BLOCKING = "10,1,2048,64,1"     # the full model's w planes on the matrix cores (W 7)
MOSAIC_W_BLOCKING64 = (16, 1, 2048, 16, 1)
CUBE_BLOCKING = "10,1,512,64,1"
METRIC = "visibilities/s fwd+adjoint NUFFT; time-to-tol cold vs learned warm start"
KERNEL_SRC = os.path.join(ROOT, "paper_2609_17636_amd", "csrc", "ivx_kernels.hip")
TRAFFIC_FILES = {"single": os.path.join(ROOT, "profiles", "k_gridmx_traffic_single.txt"),
                 "cube": os.path.join(ROOT, "profiles", "k_gridmx_traffic_cube.txt")}


# ------------------------------------------------------------------ algorithmic bytes

def grid_bytes_per_block(n_fine: int, real_bytes: int = 4) -> int:
    """Fine-grid bytes the fused degrid/residual/spread stage moves per (pointing, channel)
    block: the forward half-plane read once and the adjoint half-plane written once (G/2
    each, G = n_f^2 complex values)."""
    return n_fine * n_fine * 2 * real_bytes


def grid_algorithmic_bytes(n_live: int, n_fine: int, n_items: int = 1, real_bytes: int = 4) -> float:
    """Per-record visibility stream (coordinates 2 x 4 B, data 2 reals, weight 1 real, read
    once) plus the grid traffic of every block."""
    return n_live * (8 + 3 * real_bytes) + n_items * grid_bytes_per_block(n_fine, real_bytes)


def grid_algorithmic_bytes_shared(n_live: int, n_total: int, n_track: int, n_fine: int, n_items: int) -> float:
    """Shared-uv spectral cube: per live visibility its data (8 B), per sample a flag bit,
    per track sample its uv and weight (12 B, once for all channels), plus the grid traffic
    of every (pointing, channel) block."""
    return n_live * 8 + n_total / 8 + n_track * 12 + n_items * grid_bytes_per_block(n_fine)


def evaluation_algorithmic_bytes(vis_bytes: float, n_items: int, n_fine: int, n_sub: int, n_chan: int,
                                 n_sky: int) -> float:
    """Whole-evaluation algorithmic bytes: the visibility stream, the fine-grid passes of the
    NUFFT pair per block ((2 + 2/sigma) G with sigma = n_f / n_sub: forward rows out and
    column pass in at G/(2 sigma) each, column pass out, gridding in and out, adjoint column
    pass in at G/2 each, adjoint rows at G/(2 sigma) twice), the sub-image traffic (sky
    gather, beam twice, gradient read-modify-write: 20 B per sub-pixel) and the sky level
    (sky read, gradient write: 8 B per pixel per channel)."""
    G = n_fine * n_fine * 8
    sigma = n_fine / n_sub
    return vis_bytes + n_items * ((2 + 2 / sigma) * G + 20 * n_sub * n_sub) + 8 * n_sky * n_sky * n_chan


def grid_kernel_name(info: dict) -> str:
    """The gridding kernel a blocking runs: the matrix-core variant for lanes = 64."""
    return "k_gridmx" if info.get("lanes") == 64 else "k_grid"


def measured_traffic(workload: str, blocking: str):
    """HBM bytes per launch of the gridding kernel from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary, or None when the kernel source or the blocking changed since it was
    taken."""
    path = TRAFFIC_FILES.get(workload)
    if not path or not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    if kv.get("kernel_source_sha256") != sha or "traffic_bytes_per_launch" not in kv:
        return None
    if kv.get("blocking") != blocking:
        return None
    return float(kv["traffic_bytes_per_launch"])


def wstack_algorithmic_bytes(n_live, winfo, info, n_sub):
    """Algorithmic HBM bytes of one full-model evaluation.  Gridding (both directions, all
    planes): each live visibility meets W_w planes; per meeting the degrid pass reads its
    coordinates (8 B) and plane coordinate (4 B) and updates its accumulator (8 B read, 8 B
    written), the spread pass reads coordinates, plane coordinate and coefficient (20 B); every
    plane's extended grid (n_items x eh x ew complex, 8 B) is read once by the degrid pass and
    written once by the spread.  The evaluation adds, per plane, the row-pass buffer written
    and read in both directions and the extended grid written by the forward column pass and
    read by the adjoint one."""
    planes, ww = winfo["planes"], winfo["w_width"]
    grid_cells = info["n_items"] * info["ext_rows"] * info["ext_cols"]
    row_cells = info["n_items"] * n_sub * info["ext_cols"]
    grid = ww * n_live * (28 + 20) + 2 * planes * grid_cells * 8
    evaluation = grid + planes * (2 * 2 * row_cells + 2 * grid_cells) * 8
    return float(grid), float(evaluation)


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


# ------------------------------------------------------------------------- timing

def blocking_of(info: dict) -> str:
    return ",".join(str(info[k]) for k in ("tile", "waves_per_block", "chunk", "lanes", "vpi"))


def measure(plan, x, steps: int, warmup: int):
    """Graph-replayed timed region, then an eager pass with events around the gridding kernel
    (its average launch duration), then a short pass with events around every stage."""
    import torch

    grad = torch.empty_like(x)
    terms = torch.zeros(4, dtype=torch.float64, device=x.device)
    for _ in range(warmup):
        plan.objective_grad(x, grad=grad, terms=terms)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.objective_grad(x, grad=grad, terms=terms)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    q_tot = terms[0].item()
    # kernel pass: the same evaluations launched one by one, events around the gridding kernel
    plan.set_timing(("grid",))
    t1 = time.perf_counter()
    for _ in range(steps):
        plan.objective_grad(x, grad=grad, terms=terms)
    torch.cuda.synchronize()
    dt_eager = time.perf_counter() - t1
    stage_ms, n_timed = plan.stage_times()
    grid_ms = stage_ms["grid"] / max(n_timed, 1)
    # stage breakdown
    plan.set_timing()
    for _ in range(min(steps, 3)):
        plan.objective_grad(x, grad=grad, terms=terms)
    torch.cuda.synchronize()
    stages, n_st = plan.stage_times()
    plan.set_timing(())
    return {"dt": dt, "ms": 1e3 * dt / steps, "ms_eager": 1e3 * dt_eager / steps, "grid_ms": grid_ms,
            "stage_ms": {k: v / max(n_st, 1) for k, v in stages.items()}, "q_tot": q_tot}


def result_line(args, n_live, m, info, workload_text, extra_cfg, kernel_alg_bytes, eval_alg_bytes, traffic):
    achieved = kernel_alg_bytes / (m["grid_ms"] * 1e-3) / 1e9
    eval_gbs = eval_alg_bytes / (m["ms"] * 1e-3) / 1e9
    cfg = {"workload": workload_text, "n_vis": n_live, "n_fine": info["n_fine"],
           "kernel_width": info["kernel_width"], "parallelism": "1 GPU",
           "blocking": {k: info[k] for k in ("tile", "waves_per_block", "chunk", "lanes", "vpi")}}
    cfg.update(extra_cfg)
    return {"metric": METRIC, "value": n_live * args.steps / m["dt"], "unit": "vis/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": m["ms"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic", "config": cfg,
            "evals_per_s": 1e3 / m["ms"], "ms_per_step_eager": m["ms_eager"],
            "stage_ms": m["stage_ms"],
            "evaluation_hbm": {"algorithmic_bytes": eval_alg_bytes, "achieved": eval_gbs, "unit": "GB/s",
                               "frac": eval_gbs / HBM_PEAK_GBS},
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": grid_kernel_name(info),
                         "kernel_ms": m["grid_ms"], "algorithmic_bytes": kernel_alg_bytes}}


# ------------------------------------------------------------------ CPU baselines

def _subsample(p, m):
    import copy

    q = copy.copy(p)
    q.uv = p.uv[:m]
    q.vis = p.vis[:m]
    q.weight = p.weight[:m]
    q.flags = None if p.flags is None else p.flags[:m]
    q.vis_offsets = np.array([0, m], dtype=np.int64)
    return q


def cpu_baseline_single(p, x, target_s=12.0):
    """FP64 oracle (direct DFT forward + explicit adjoint + Laplacian) on a bounded sample of
    the single-pointing workload: the first M_s visibilities, M_s grown until ~target_s of
    CPU work."""
    import oracle

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


def cpu_baseline_cube(p, x, n_live_total, k=17, c=64):
    """FP64 oracle on one whole (pointing, channel) block of the cube -- every live
    visibility of pointing k in channel c through the direct DFT and its explicit adjoint, the
    reprojection and its transpose, plus channel c's Laplacian and single-dish terms -- at the
    benchmark's sky.  The oracle's cost is the direct DFT's, M * n_sub^2 per direction, and
    n_sub is the same for every block, so the full evaluation is extrapolated in proportion
    to the live visibilities (labelled as such)."""
    import oracle

    q = p.block_problem(k, c, x=x)
    live = int((q.flags == 0).sum())
    t0 = time.perf_counter()
    oracle.objective_grad(q, q.x_true)
    dt = time.perf_counter() - t0
    rate = live / dt
    return {"value": rate, "unit": "vis/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"one full (pointing, channel) block of the cube (pointing {k}, channel {c}: "
                      f"{live} live visibilities, {p.n_sub}^2 sub-image, {p.n_sky}^2 channel sky with its Laplacian "
                      f"and single-dish terms), one FP64 objective+gradient evaluation in {dt:.1f} s",
            "seconds": dt, "extrapolated_full_evaluation_s": n_live_total / rate}


# ----------------------------------------------------------------------- workloads

def run_single(args):
    """512^2 sky at 7 arcsec (k^-3 log-normal, 0-50 K), one pointing, 630 baselines x 1000
    samples = 630,000 visibilities, lambda_r = 1e-2; data = HIP forward of the true sky plus
    1% noise."""
    import torch

    import synth
    from paper_2609_17636_amd import Plan

    dev = torch.device("cuda:0")
    p = synth.config_c2(2001)
    print(f"# workload {p.name}: N={p.n_sky} vis={p.n_vis}", file=sys.stderr, flush=True)
    plan = Plan.from_problem(p)
    p.vis = np.zeros(p.n_vis, dtype=np.complex64)
    plan.set_problem_data(p)
    mv = plan.forward(torch.tensor(p.x_true, dtype=torch.float32, device=dev)).double().cpu().numpy()
    synth.attach_data(p, mv[:, 0] + 1j * mv[:, 1])
    plan.set_problem_data(p)
    if args.autotune:
        plan.autotune(2000.0)
    else:
        plan.set_blocking(*[int(v) for v in (args.blocking or SINGLE_BLOCKING).split(",")])
    info = plan.info()
    print(f"# plan {info}", file=sys.stderr, flush=True)
    rng = np.random.default_rng(0)
    xh = rng.uniform(0, 50, size=p.x_true.shape)
    x = torch.tensor(xh, dtype=torch.float32, device=dev)
    m = measure(plan, x, args.steps, args.warmup)
    n_live = info["n_live_vis"]
    alg = grid_algorithmic_bytes(n_live, info["n_fine"])
    ev = evaluation_algorithmic_bytes(n_live * 20, 1, info["n_fine"], p.n_sub, 1, p.n_sky)
    out = result_line(args, n_live, m, info,
                      "single-pointing 512x512 sky (7 arcsec, k^-3 log-normal 0-50 K), 630 baselines x 1000 "
                      "samples = 630,000 visibilities, lambda_r=1e-2", {"n_sky": p.n_sky},
                      alg, ev, measured_traffic("single", blocking_of(info)))
    print(f"# {m['ms']:.4f} ms/eval (graph), {m['ms_eager']:.4f} eager, grid {m['grid_ms']:.4f} ms/launch, "
          f"Q_tot={m['q_tot']:.6e}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_single(p, xh, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def run_mosaic(args, w_term: bool = False):
    """The 36-pointing mosaic: 1024^2 sky at 30", 6 x 6 hex of 1 deg beams, 384^2
    sub-images, 1400-2000 samples x 630 baselines per pointing with 0-30% flags (about 34 M
    live visibilities), 64 x 64 single-dish map, lambda_r = 1e-2, lambda_s = 1.  Data from the
    FP64 HIP forward of the true sky plus 1% noise per pointing.  w_term: the full model of
    Eq. vis (w-stacked; the sub-images reach 2.3 deg from their phase centres)."""
    import torch

    import synth
    from paper_2609_17636_amd import Plan

    dev = torch.device("cuda:0")
    p = synth.config_c3(w_term=w_term)
    synth.attach_sd_level(p)
    p.vis = np.zeros(p.n_vis, dtype=np.complex64)
    print(f"# workload {p.name}: N={p.n_sky} vis={p.n_vis} live={int((p.flags == 0).sum())}", file=sys.stderr,
          flush=True)
    plan64 = Plan.from_problem(p, precision="f64")
    plan64.set_problem_data(p)
    if w_term:
        plan64.set_blocking(*MOSAIC_W_BLOCKING64)
        plan64.set_w(p.w)
    mv = plan64.forward(torch.tensor(p.x_true, dtype=torch.float64, device=dev)).cpu().numpy()
    del plan64
    synth.attach_data(p, mv[:, 0] + 1j * mv[:, 1])
    plan = Plan.from_problem(p)
    plan.set_problem_data(p)
    if args.blocking:
        plan.set_blocking(*[int(v) for v in args.blocking.split(",")])
    elif w_term:
        plan.set_blocking(*[int(v) for v in MOSAIC_W_BLOCKING.split(",")])
    else:
        plan.autotune(3000.0)
    if w_term:
        plan.set_w(p.w)
        print(f"# w planes {plan.w_info()}", file=sys.stderr, flush=True)
    info = plan.info()
    print(f"# plan {info}", file=sys.stderr, flush=True)
    rng = np.random.default_rng(0)
    x = torch.tensor(rng.uniform(0, 50, size=p.x_true.shape), dtype=torch.float32, device=dev)
    m = measure(plan, x, args.steps, args.warmup)
    n_live = info["n_live_vis"]
    alg = grid_algorithmic_bytes(n_live, info["n_fine"], n_items=info["n_items"])
    ev = evaluation_algorithmic_bytes(n_live * 20, info["n_items"], info["n_fine"], p.n_sub, 1, p.n_sky)
    if w_term:
        alg, ev = wstack_algorithmic_bytes(n_live, plan.w_info(), info, p.n_sub)
    out = result_line(args, n_live, m, info,
                      "36-pointing mosaic, 1024^2 sky at 30 arcsec, 384^2 sub-images, "
                      f"{n_live} live visibilities, single-dish 64x64, lambda_r=1e-2, lambda_s=1"
                      + (", full model of Eq. vis (w-stacked)" if w_term else ""),
                      {"n_sky": p.n_sky}, alg, ev, None)
    if w_term:
        out["roofline"]["kernel"] = (grid_kernel_name(info) + " w-plane modes (all planes, both directions)")
        out["config"]["w_planes"] = plan.w_info()
    print(f"# {m['ms']:.4f} ms/eval, grid {m['grid_ms']:.4f} ms/launch, Q_tot={m['q_tot']:.6e}", file=sys.stderr,
          flush=True)
    print(json.dumps(out), flush=True)


def run_cube(args):
    """The spectral cube (module docstring).  Data: unit-variance complex noise per
    visibility and a constant-level single-dish map with 1% noise (the cost does not depend
    on the values); the sky is uniform 0-50 K."""
    import torch

    import synth
    from paper_2609_17636_amd import Plan

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    p = synth.config_c4(with_field=False)
    p.lambda_nu = float(args.lambda_nu)
    synth.attach_sd_level(p)
    n_total, n_track = p.n_vis, int(p.pt_offsets[-1])
    print(f"# workload {p.name}: N={p.n_sky} C={p.n_chan} P={p.n_point} vis={n_total} "
          f"({time.perf_counter() - t0:.1f} s to generate)", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    blocking = [int(v) for v in (args.blocking or CUBE_BLOCKING).split(",")]
    plan = Plan.from_problem(p, tile=blocking[0])
    plan.set_cube_data(p)
    if args.autotune:
        plan.autotune(3000.0)
    else:
        plan.set_blocking(*blocking)
    torch.cuda.synchronize()
    info = plan.info()
    print(f"# plan in {time.perf_counter() - t0:.1f} s: {info}", file=sys.stderr, flush=True)
    rng = np.random.default_rng(0)
    xh = rng.uniform(0, 50, size=(p.n_chan, p.n_sky, p.n_sky)).astype(np.float32)
    x = torch.tensor(xh, device=dev)
    m = measure(plan, x, args.steps, args.warmup)
    n_live = info["n_live_vis"]
    alg = grid_algorithmic_bytes_shared(n_live, n_total, n_track, info["n_fine"], info["n_items"])
    vis_bytes = n_live * 8 + n_total / 8 + n_track * 12
    ev = evaluation_algorithmic_bytes(vis_bytes, info["n_items"], info["n_fine"], p.n_sub, p.n_chan, p.n_sky)
    out = result_line(args, n_live, m, info,
                      "spectral cube, 128 channels x 36 pointings, 1024^2 sky at 30 arcsec, 384^2 sub-images, "
                      f"shared uv per pointing, {n_live} live visibilities, single-dish 64x64 per channel, "
                      "lambda_r=1e-2, lambda_s=1" + (f", lambda_nu={p.lambda_nu:g}" if p.lambda_nu else ""),
                      {"n_sky": p.n_sky, "n_chan": p.n_chan, "n_point": p.n_point, "device_bytes": info["device_bytes"]},
                      alg, ev, measured_traffic("cube", blocking_of(info)))
    print(f"# {m['ms']:.2f} ms/eval (graph), {m['ms_eager']:.2f} eager, grid {m['grid_ms']:.2f} ms/launch, "
          f"Q_tot={m['q_tot']:.6e}, stages {json.dumps(m['stage_ms'])}", file=sys.stderr, flush=True)
    del plan, x
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_cube(p, xh, n_live)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="single-pointing oracle sample budget")
    ap.add_argument("--copy-probe", action="store_true", help="run the counter calibration copy only")
    ap.add_argument("--blocking", default=None,
                    help="tile,waves,chunk,lanes,vpi of the gridding kernel (default: the autotuner's choice "
                         f"for the workload, recorded: cube {CUBE_BLOCKING}, single {SINGLE_BLOCKING})")
    ap.add_argument("--autotune", action="store_true", help="run the plan autotuner instead of --blocking")
    ap.add_argument("--lambda-nu", type=float, default=0.0,
                    help="cube only: weight of the spectral smoothness term (0: the paper's independent channels)")
    ap.add_argument("--workload", default="cube", choices=("cube", "single", "mosaic", "mosaic-w"),
                    help="cube: the 128-channel spectral cube (default, the largest single-GPU "
                         "configuration); single: the 512^2 single-pointing problem; mosaic: the "
                         "one-channel 36-pointing mosaic; mosaic-w: the same with the full model of "
                         "Eq. vis")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe(args.steps)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: the library runs on one "
              f"GPU (sharding channels and pointings across GPUs is described, not implemented)", file=sys.stderr)
        sys.exit(2)
    {"cube": run_cube, "single": run_single, "mosaic": run_mosaic,
     "mosaic-w": lambda a: run_mosaic(a, w_term=True)}[args.workload](args)


if __name__ == "__main__":
    main()
