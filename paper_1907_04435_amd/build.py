"""Build libsa.so (the HIP library for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsa.so")
OBJ = os.path.join(HERE, "_build")
SOURCES = ["api.cpp", "sunpath.cpp", "bvh.hip", "accumulate.hip", "grad.hip", "reduce.hip", "sam.hip", "peak.hip"]
ARCH = "gfx950"

# Device code: never emit packed-FP32 instructions (disabled outright for
# this target).
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# Kernel sources only: no NaN propagation semantics and IEEE mode off.  In
# IEEE mode every fminf/fmaxf on a loaded value first quiets signalling
# NaNs (an extra v_max per operand: ~28% of the accrual kernel's VALU
# code).  In these kernels a NaN can only arise in a temporary that a
# select then discards (0 * inf in a parallel edge or a flat clip edge), so
# nothing depends on NaN semantics.  Host sources (input validation with
# isfinite) keep full IEEE semantics.
KERNEL_FLAGS = ["-fno-honor-nans", "-mno-amdgpu-ieee"]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    hipcc = _hipcc()
    common = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-result",
              "-I", os.path.join(HERE, "..", "include")]
    objs = []

    def compile_one(src):
        obj = os.path.join(OBJ, src + ".o")
        cmd = [hipcc, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj] + common + DEVICE_FLAGS
        if src.endswith(".hip"):
            cmd += KERNEL_FLAGS
        r = subprocess.run(cmd, capture_output=True, text=True)
        out = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                        if "packed-fp32-ops" not in l and "warning generated" not in l
                        and "warnings generated" not in l)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{out}")
        if verbose and out.strip():
            print(out, file=sys.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
