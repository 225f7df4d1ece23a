"""Summarise a rocprofv3 results database (kernel trace, optionally PMC counters).

    python -m paper_2609_17636_amd.profile_summary RESULTS.db [--last N] [--kernel REGEX]
    python -m paper_2609_17636_amd.profile_summary --traffic FETCH.db WRITE.db COPY_FETCH.db \
        COPY_WRITE.db --kernel REGEX --last N [--note TEXT]

Per kernel: dispatch count, average / min / max duration (us) and share of the total,
over all dispatches or over the last N dispatches of each kernel (the timed region of
bench.py, which launches every evaluation kernel once per step after all set-up and
autotuning).  With PMC data present, the per-dispatch average of every counter is
printed too (FETCH_SIZE / WRITE_SIZE are in KiB per dispatch).
"""
from __future__ import annotations

import argparse
import re
import sqlite3


def _short(name: str) -> str:
    return re.sub(r"\(.*", "", name.replace("(anonymous namespace)::", ""))


def kernel_rows(db: str):
    con = sqlite3.connect(db)
    cols = [r[1] for r in con.execute("pragma table_info(kernels)")]
    ci = {c: i for i, c in enumerate(cols)}
    out = []
    for r in con.execute("select * from kernels order by start"):
        out.append((_short(r[ci["name"]]), r[ci["start"]], r[ci["end"]], r[ci["dispatch_id"]]))
    return con, out


def pmc_by_dispatch(con):
    try:
        cols = [r[1] for r in con.execute("pragma table_info(pmc_events)")]
    except sqlite3.Error:
        return {}
    if not cols:
        return {}
    ci = {c: i for i, c in enumerate(cols)}
    res = {}
    name_col = "counter_name" if "counter_name" in ci else ("name" if "name" in ci else None)
    val_col = "value" if "value" in ci else ("counter_value" if "counter_value" in ci else None)
    disp_col = "dispatch_id" if "dispatch_id" in ci else None
    if not (name_col and val_col and disp_col):
        return {}
    for r in con.execute("select * from pmc_events"):
        d = res.setdefault(r[ci[disp_col]], {})
        d[r[ci[name_col]]] = d.get(r[ci[name_col]], 0.0) + float(r[ci[val_col]])
    return res


def summarise(db: str, last: int = 0, kernel: str = "") -> str:
    con, rows = kernel_rows(db)
    pmc = pmc_by_dispatch(con)
    by = {}
    for name, t0, t1, disp in rows:
        if kernel and not re.search(kernel, name):
            continue
        by.setdefault(name, []).append((t1 - t0, disp))
    if last:
        by = {k: v[-last:] for k, v in by.items()}
    total = sum(d for v in by.values() for d, _ in v) or 1
    lines = [f"{'kernel':62s} {'calls':>6s} {'avg_us':>9s} {'min_us':>9s} {'max_us':>9s} {'share%':>7s}"]
    for name, v in sorted(by.items(), key=lambda kv: -sum(d for d, _ in kv[1])):
        ds = [d for d, _ in v]
        lines.append(f"{name[:62]:62s} {len(ds):6d} {sum(ds) / len(ds) / 1e3:9.2f} {min(ds) / 1e3:9.2f} "
                     f"{max(ds) / 1e3:9.2f} {100 * sum(ds) / total:7.2f}")
        counters = {}
        for _, disp in v:
            for c, val in pmc.get(disp, {}).items():
                counters.setdefault(c, []).append(val)
        for c, vals in sorted(counters.items()):
            lines.append(f"    {c}: {sum(vals) / len(vals):.1f} per dispatch ({len(vals)} dispatches)")
    return "\n".join(lines)


def counter_avg(db: str, kernel: str, counter: str, last: int = 0) -> float:
    """Per-dispatch average of one PMC counter over the (last N) dispatches of the kernels
    matching `kernel`."""
    con, rows = kernel_rows(db)
    pmc = pmc_by_dispatch(con)
    vals = [pmc[d][counter] for name, _, _, d in rows if re.search(kernel, name) and counter in pmc.get(d, {})]
    if last:
        vals = vals[-last:]
    if not vals:
        raise SystemExit(f"no {counter} values for /{kernel}/ in {db}")
    return sum(vals) / len(vals)


COPY_BYTES = 1 << 30   # bytes read and written by one dispatch of bench.py --copy-probe


def traffic_report(fetch_db, write_db, copy_fetch_db, copy_write_db, kernel, last, note="", blocking="") -> str:
    """HBM bytes per launch of `kernel` from FETCH_SIZE / WRITE_SIZE (KiB per dispatch),
    each scaled by the factor that makes the same counter read the known 1 GiB of the
    calibration copy."""
    import hashlib
    import os

    f_k = counter_avg(fetch_db, kernel, "FETCH_SIZE", last)
    w_k = counter_avg(write_db, kernel, "WRITE_SIZE", last)
    f_c = counter_avg(copy_fetch_db, "copyBuffer", "FETCH_SIZE")
    w_c = counter_avg(copy_write_db, "copyBuffer", "WRITE_SIZE")
    ff = COPY_BYTES / (f_c * 1024.0)
    fw = COPY_BYTES / (w_c * 1024.0)
    fetch_b = f_k * 1024.0 * ff
    write_b = w_k * 1024.0 * fw
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "ivx_kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    out = [f"# HBM traffic of /{kernel}/ per launch (rocprofv3 PMC, last {last} dispatches)"]
    if note:
        out.append(f"# {note}")
    if blocking:
        out.append(f"blocking: {blocking}")
    out += [f"kernel: {kernel}",
            f"fetch_kib_per_dispatch: {f_k:.1f}",
            f"write_kib_per_dispatch: {w_k:.1f}",
            f"copy_fetch_kib_per_dispatch: {f_c:.1f}",
            f"copy_write_kib_per_dispatch: {w_c:.1f}",
            f"fetch_factor: {ff:.4f}",
            f"write_factor: {fw:.4f}",
            f"fetch_bytes_per_launch: {fetch_b:.0f}",
            f"write_bytes_per_launch: {write_b:.0f}",
            f"traffic_bytes_per_launch: {fetch_b + write_b:.0f}",
            f"kernel_source_sha256: {sha}"]
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("db", nargs="?")
    ap.add_argument("--last", type=int, default=0)
    ap.add_argument("--kernel", default="")
    ap.add_argument("--traffic", nargs=4, metavar=("FETCH_DB", "WRITE_DB", "COPY_FETCH_DB", "COPY_WRITE_DB"))
    ap.add_argument("--note", default="")
    ap.add_argument("--blocking", default="", help="gridding blocking the counters were taken with")
    a = ap.parse_args()
    if a.traffic:
        print(traffic_report(*a.traffic, kernel=a.kernel, last=a.last, note=a.note,
                             blocking=a.blocking))
    else:
        print(summarise(a.db, a.last, a.kernel))


if __name__ == "__main__":
    main()
