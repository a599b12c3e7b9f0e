"""Build libcrk.so (all HIP kernels + C ABI) for gfx950 with hipcc, in-tree.

Usage: python -m paper_2502_03091_amd.build  (or build() from Python).
Every source is compiled on each call; objects go to _build/ beside this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libcrk.so")

SOURCES = [
    "geometry.hip",
    "clover.hip",
    "dslash.hip",
    "blas.hip",
    "svd.hip",
    "galerkin.hip",
    "coarse.hip",
    "transfer.hip",
    "gcr.hip",
    "mg.hip",
    "solver.hip",
    "lattice.cpp",
    "capi.cpp",
    "capi_mg.cpp",
    "server.cpp",
    "pool.cpp",
    "noalloc.hip",
]

ARCH = os.environ.get("CRK_OFFLOAD_ARCH", "gfx950")
FLAGS = [
    "-O3",
    "-std=c++17",
    "-fPIC",
    f"--offload-arch={ARCH}",
    # packed fp32 instructions are kept out of every device kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"),
]


def _hipcc():
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(h):
        raise RuntimeError("hipcc not found: the crk library needs ROCm's hipcc")
    return h


def _compile(src, obj, extra):
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [_hipcc(), *FLAGS, *extra, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    return r.stderr


def build(verbose=False, jobs=None, extra=()):
    out = os.path.join(HERE, "_build")
    os.makedirs(out, exist_ok=True)
    objs = []
    jobs = jobs or min(8, len(SOURCES))
    with cf.ThreadPoolExecutor(jobs) as ex:
        futs = {}
        for s in SOURCES:
            o = os.path.join(out, os.path.splitext(s)[0] + ".o")
            objs.append(o)
            futs[ex.submit(_compile, s, o, list(extra))] = s
        for f in cf.as_completed(futs):
            msg = f.result()
            if verbose and msg.strip():
                print(f"[{futs[f]}]\n{msg}", file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-pthread", "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
