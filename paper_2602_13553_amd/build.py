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


# The host-side debug build: the library's host code (parameter checks,
# layouts, atom ordering, batch plans) under AddressSanitizer and
# UndefinedBehaviorSanitizer; the device code is built as usual.  The
# sanitizer runtime is not linked in: the process that loads the library
# preloads clang's shared ASan runtime (which carries the UBSan handlers).
LIB_HOST_SAN = os.path.join(HERE, "libpimd_hostsan.so")
HOST_SAN_FLAGS = ["-Xarch_host", "-fsanitize=address,undefined",
                  "-Xarch_host", "-fno-sanitize-recover=all",
                  "-Xarch_host", "-fno-omit-frame-pointer"]


def build(verbose: bool = False, host_sanitize: bool = False) -> str:
    """Always recompiles (the 'does it build' check); returns the library path.
    host_sanitize: build LIB_HOST_SAN instead (see HOST_SAN_FLAGS)."""
    suffix = ".hostsan.o" if host_sanitize else ".o"
    objs, cmds = [], []
    for s in SOURCES:
        obj = os.path.join(CSRC, os.path.splitext(s)[0] + suffix)
        cmds.append([hipcc(), *HIP_FLAGS, *(HOST_SAN_FLAGS if host_sanitize else []),
                     "-I", os.path.join(ROOT, "include"), "-c", os.path.join(CSRC, s), "-o", obj])
        objs.append(obj)
    # the translation units compile in parallel (one hipcc each)
    procs = []
    for cmd in cmds:
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
    failed = [c for c, pr in zip(cmds, procs) if pr.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    out = LIB_HOST_SAN if host_sanitize else LIB
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    for o in objs:
        os.remove(o)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
