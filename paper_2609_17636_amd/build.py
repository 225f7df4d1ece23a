"""Build the gfx950 shared libraries in-tree with hipcc.

libivx.so      : ivx_real = float (the product build)
libivx_f64.so  : ivx_real = double (FP64 test build, same symbols)
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
SOURCES = ["ivx_api.hip", "ivx_build.hip", "ivx_kernels.hip", "ivx_unet.hip", "ivx_lbfgsb.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

LIBS = {"f32": "libivx.so", "f64": "libivx_f64.so"}


def lib_path(precision: str = "f32") -> str:
    return os.path.join(HERE, LIBS[precision])


def build(precisions=("f32", "f64"), verbose: bool = False) -> list:
    out = []
    for prec in precisions:
        target = lib_path(prec)
        tmp = target + ".tmp"
        cmd = [HIPCC, "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wno-unused-command-line-argument", "-I", INCLUDE, "-I", CSRC]
        if prec == "f64":
            cmd.append("-DIVX_REAL_DOUBLE")
        cmd += [os.path.join(CSRC, s) for s in SOURCES] + ["-o", tmp]
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
