"""Build libionic_sdc.so for gfx950 with hipcc, in-tree.

Every HIP translation unit is compiled with packed-FP32 instructions
disabled (-Xclang -target-feature -Xclang -packed-fp32-ops); the model
kernels compile in parallel, then hipcc links the shared library.  The device
assembly of every unit is checked for a known miscompilation (spill code ahead
of an execution-mask restore, codegen_check.py) before linking.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

try:
    from . import codegen_check
except ImportError:  # run as a script
    import codegen_check

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIBDIR = os.path.join(PKG, "_lib")
OBJDIR = os.path.join(LIBDIR, "obj")
LIBNAME = "libionic_sdc.so"
LIBPATH = os.path.join(LIBDIR, LIBNAME)
# rate microbenchmarks of the units the step kernels are bound by (measurement
# support for bench.py, a library of its own)
MB_SOURCES = ["microbench.hip"]
MB_LIBPATH = os.path.join(LIBDIR, "libionic_microbench.so")

STEP_FP64 = ["kernels_%s_fp64%s.hip" % (m, p) for m in ("tt06", "lr91") for p in ("", "_ros2", "_rl")]
STEP_MIXED = ["kernels_%s_mixed%s.hip" % (m, p) for m in ("tt06", "lr91") for p in ("", "_ros2", "_rl")]
# slowest first, so the parallel build ends sooner
SOURCES = STEP_FP64 + STEP_MIXED + ["kernels_tt06.hip", "kernels_lr91.hip", "kernels_test.hip",
                                    "control.hip", "diffusion.hip", "elliptic.hip", "multigrid.hip",
                                    "implicit.hip",
                                    "multigrid_plan.cpp",
                                    "ionic.cpp"]
# per-source optimisation level (default -O3)
OPT = {}
# the mixed-precision step kernels may reassociate fp arithmetic (NaN/Inf
# semantics kept, so non-finite states are still detected); results move at
# the rounding level only, far below the mixed path's tolerance
EXTRA = {s: ["-fassociative-math", "-fno-signed-zeros", "-fno-trapping-math"] for s in STEP_MIXED}
# the step kernels run at the register limit (one wavefront per SIMD, spills in
# fp64); the scheduler's own register-pressure trackers place fewer spill and
# register-copy instructions there (the same results bit for bit; TT06 fp64
# pass 1.58 -> 1.47 s, mixed 243 -> 240 ms on the 1e6-vertex slab)
for _s in STEP_FP64 + STEP_MIXED + ["implicit.hip"]:
    EXTRA[_s] = EXTRA.get(_s, []) + ["-mllvm", "-amdgpu-use-amdgpu-trackers"]
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
    stem = os.path.splitext(src)[0]
    obj = os.path.join(OBJDIR, stem + ".o")
    # -save-temps keeps the device assembly of this very compile for the check below
    cmd = ([_hipcc(), "-x", "hip", OPT.get(src, "-O3")] + FLAGS + EXTRA.get(src, []) + extra
           + ["-save-temps=obj", "-c", os.path.join(CSRC, src), "-o", obj])
    r = subprocess.run(cmd, capture_output=True, text=True, cwd=OBJDIR)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), r.stderr[-6000:]))
    if src.endswith(".hip"):
        asm = os.path.join(OBJDIR, "%s-hip-amdgcn-amd-amdhsa-%s.s" % (stem, ARCH))
        if not os.path.exists(asm):
            raise RuntimeError("device assembly of %s not found at %s" % (src, asm))
        found = codegen_check.check_file(asm)
        if found:
            lines = "\n".join("  %s %s line %d: %s" % f for f in found[:20])
            raise RuntimeError(
                "%s: %d lane-masked vector writes placed before the execution-mask restore of "
                "a divergent join (a miscompilation that loses values of masked lanes):\n%s"
                % (src, len(found), lines))
    return obj


def build(jobs: int = 8, extra_flags=(), verbose: bool = True) -> str:
    """Compile every source and link the shared library; returns its path."""
    os.makedirs(OBJDIR, exist_ok=True)
    extra = list(extra_flags)
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(lambda s: _compile(s, extra), SOURCES + MB_SOURCES))
    for path, lib_objs in ((LIBPATH, objs[:len(SOURCES)]), (MB_LIBPATH, objs[len(SOURCES):])):
        tmp = path + ".tmp"
        cmd = [_hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH] + lib_objs + ["-o", tmp]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), r.stderr[-6000:]))
        os.replace(tmp, path)
        if verbose:
            print("built", path, file=sys.stderr)
    return LIBPATH


if __name__ == "__main__":
    build(jobs=int(os.environ.get("MAX_JOBS", "4")))
