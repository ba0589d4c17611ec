"""Build libgb.so (HIP kernels for gfx950 + host setup) in-tree.

    python -m paper_2607_00199_amd.build

Device code is compiled with packed FP32 instructions disabled (the host pass
warns that it does not know the feature; that warning is harmless).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(ROOT, "_build")
OUT = os.path.join(HERE, "libgb.so")
ARCH = os.environ.get("GB_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include")]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-I", os.path.join(ROOT, "include")]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError(f"build step failed: {cmd[0]} ... {cmd[-1]}")
    return r


def build(verbose: bool = False) -> str:
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    cxx = shutil.which("g++") or "c++"
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    objs = []

    def cost(name: str) -> int:
        # heaviest translation units first (tetrahedra, high orders, FP64) so
        # the longest compiles do not start last
        parts = name.replace(".hip", "").split("_")
        if name.startswith("gb_shape_") and len(parts) == 5:
            dim, order, prec = int(parts[2]), int(parts[3]), parts[4]
            return -(100 * dim + 10 * order + (1 if prec == "f64" else 0))
        return 0

    for name in sorted(os.listdir(CSRC), key=lambda n: (cost(n), n)):
        src = os.path.join(CSRC, name)
        obj = os.path.join(BUILD, name + ".o")
        if name.endswith(".hip"):
            jobs.append([hipcc, *HIP_FLAGS, "-c", src, "-o", obj])
        elif name.endswith(".cpp"):
            jobs.append([cxx, *HOST_FLAGS, "-c", src, "-o", obj])
        else:
            continue
        objs.append(obj)
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        list(ex.map(_run, jobs))
    tmp = OUT + ".tmp"
    _run([hipcc, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs])
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
