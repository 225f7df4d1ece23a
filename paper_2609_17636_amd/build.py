"""Build the gfx950 shared libraries in-tree with hipcc.

libivx.so      : ivx_real = float (the product build)
libivx_f64.so  : ivx_real = double (FP64 test build, same symbols)

Every (precision, source) pair is compiled to its own object in parallel, then each
library is linked from its objects.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(HERE, "_build")
SOURCES = ["ivx_api.hip", "ivx_build.hip", "ivx_kernels.hip", "ivx_unet.hip", "ivx_lbfgsb.hip", "ivx_dataproc.hip", "ivx_wstack.hip", "ivx_sort.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument", "-I", INCLUDE, "-I", CSRC]

LIBS = {"f32": "libivx.so", "f64": "libivx_f64.so"}


def lib_path(precision: str = "f32") -> str:
    return os.path.join(HERE, LIBS[precision])


def _defines(prec: str) -> list:
    return ["-DIVX_REAL_DOUBLE"] if prec == "f64" else []


def _compile(prec: str, src: str, verbose: bool) -> str:
    obj = os.path.join(OBJDIR, f"{os.path.splitext(src)[0]}_{prec}.o")
    cmd = [HIPCC] + FLAGS + _defines(prec) + ["-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    return obj


def build(precisions=("f32", "f64"), verbose: bool = False, jobs: int = 0) -> list:
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = jobs or min(16, os.cpu_count() or 4)
    pairs = [(p, s) for p in precisions for s in SOURCES]
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda ps: _compile(ps[0], ps[1], verbose), pairs))
    out = []
    for prec in precisions:
        target = lib_path(prec)
        tmp = target + ".tmp"
        mine = [o for (p, _), o in zip(pairs, objs) if p == prec]
        cmd = [HIPCC, "--offload-arch=gfx950", "-fPIC", "-shared"] + mine + ["-o", tmp]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        subprocess.run(cmd, check=True)
        os.replace(tmp, target)
        out.append(target)
    return out


if __name__ == "__main__":
    prec = sys.argv[1:] or ["f32", "f64"]
    for p in build(prec, verbose=True):
        print(p)
