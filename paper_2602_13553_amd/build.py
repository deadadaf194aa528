"""Compile libpimd.so for gfx950 with hipcc (cross-compiles without a GPU)."""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpimd.so")
SOURCES = ["pimd_kernels.hip", "pimd_fused_mfma.hip", "pimd_npt.hip", "pimd_boson.hip",
           "pimd_api.hip"]

# Packed FP32 instructions (v_pk_*_f32) are disabled for every HIP translation
# unit.  The host pass prints "'-packed-fp32-ops' is not a recognized feature
# for this target": it has no such feature and ignores it.  The gfx950 device
# pass honours it: a float2 multiply-add kernel compiles to v_pk_fma_f32
# without the flag and to none with it (tests/test_build_flags.py).
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    """Always recompiles (the 'does it build' check); returns the library path."""
    objs = []
    for s in SOURCES:
        obj = os.path.join(CSRC, os.path.splitext(s)[0] + ".o")
        cmd = [hipcc(), *HIP_FLAGS, "-I", os.path.join(ROOT, "include"), "-c",
               os.path.join(CSRC, s), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
