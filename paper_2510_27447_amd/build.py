"""Build libionic_sdc.so for gfx950 with hipcc, in-tree.

Every HIP translation unit is compiled with packed-FP32 instructions
disabled (-Xclang -target-feature -Xclang -packed-fp32-ops); the model
kernels compile in parallel, then hipcc links the shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIBDIR = os.path.join(PKG, "_lib")
OBJDIR = os.path.join(LIBDIR, "obj")
LIBNAME = "libionic_sdc.so"
LIBPATH = os.path.join(LIBDIR, LIBNAME)

SOURCES = ["kernels_tt06_fp64.hip", "kernels_tt06.hip", "kernels_lr91_fp64.hip",
           "kernels_lr91.hip", "kernels_test.hip", "ionic.cpp"]
# per-source optimisation level (default -O3); the double-precision step
# kernels of the cell models are built at -O1, where their code is exact
# (see the headers of those files)
OPT = {"kernels_tt06_fp64.hip": "-O1", "kernels_lr91_fp64.hip": "-O1"}
# the mixed-precision step kernels may reassociate fp arithmetic (NaN/Inf
# semantics kept, so non-finite states are still detected); results move at
# the rounding level only, far below the mixed path's tolerance
EXTRA = {s: ["-fassociative-math", "-fno-signed-zeros", "-fno-trapping-math"]
         for s in ("kernels_tt06.hip", "kernels_lr91.hip")}
ARCH = os.environ.get("IONIC_OFFLOAD_ARCH", "gfx950")
FLAGS = [
    "--offload-arch=" + ARCH, "-std=c++20", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + INCLUDE, "-I" + CSRC,
]


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src, extra):
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = ([_hipcc(), "-x", "hip", OPT.get(src, "-O3")] + FLAGS + EXTRA.get(src, []) + extra
           + ["-c", os.path.join(CSRC, src), "-o", obj])
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), r.stderr[-6000:]))
    return obj


def build(jobs: int = 6, extra_flags=(), verbose: bool = True) -> str:
    """Compile every source and link the shared library; returns its path."""
    os.makedirs(OBJDIR, exist_ok=True)
    extra = list(extra_flags)
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(lambda s: _compile(s, extra), SOURCES))
    tmp = LIBPATH + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH] + objs + ["-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), r.stderr[-6000:]))
    os.replace(tmp, LIBPATH)
    if verbose:
        print("built", LIBPATH, file=sys.stderr)
    return LIBPATH


if __name__ == "__main__":
    build(jobs=int(os.environ.get("MAX_JOBS", "4")))
