"""Build libgraf_af.so (HIP, gfx950) in-tree.

Every translation unit compiles in parallel with hipcc; kernel variants are
separate units (af_variant.hip with -DGRAF_VARIANT=k) so the large templated
kernels build side by side.  Packed FP32 instructions are switched off for all
device code.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libgraf_af.so")
N_VARIANTS = 6

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include")]


def _units():
    units = [("af_api.hip", [], "af_api.o"),
             ("af_reduce.hip", [], "af_reduce.o"),
             ("mlp_kernels.hip", [], "mlp_kernels.o"),
             ("af_cross.hip", [], "af_cross.o"),
             ("af_union.hip", [], "af_union.o")]
    for v in range(N_VARIANTS):
        units.append(("af_variant.hip", ["-DGRAF_VARIANT=%d" % v], "af_variant%d.o" % v))
    return [u for u in units if os.path.exists(os.path.join(CSRC, u[0]))]


def _compile(unit):
    src, extra, obj = unit
    out = os.path.join(BUILD, obj)
    cmd = [HIPCC] + FLAGS + extra + ["-c", os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [ln for ln in (r.stdout + r.stderr).splitlines()
            if ln.strip() and "packed-fp32-ops" not in ln]
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, "\n".join(msgs)))
    return out


def build(jobs=None, verbose=True):
    """Compile every unit and link libgraf_af.so; returns the library path."""
    if shutil.which(HIPCC) is None and not os.path.exists(HIPCC):
        raise RuntimeError("hipcc not found at %s" % HIPCC)
    os.makedirs(BUILD, exist_ok=True)
    units = _units()
    jobs = jobs or min(len(units), max(1, min(16, os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, units))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB, file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build()
