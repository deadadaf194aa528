"""The library's HIP flags keep packed FP32 instructions out of device code.

Compiles a float2 multiply-add kernel for gfx950 with and without the
library's flags and reads the device assembly (CPU only; needs hipcc)."""
from __future__ import annotations

import os
import re
import subprocess
import tempfile

import pytest

from paper_2602_13553_amd import build as pbuild

SRC = r"""
#include <hip/hip_runtime.h>
__global__ void k(float2 *a, const float2 *b, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        float2 x = a[i], y = b[i];
        x.x = x.x * y.x + 1.0f;
        x.y = x.y * y.y + 1.0f;
        a[i] = x;
    }
}
"""


def _device_asm(flags):
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "k.hip")
        out = os.path.join(d, "k.s")
        with open(src, "w") as fh:
            fh.write(SRC)
        subprocess.run([pbuild.hipcc(), *flags, "--cuda-device-only", "-S", src, "-o", out],
                       check=True, capture_output=True)
        with open(out) as fh:
            return fh.read()


def test_no_packed_fp32_with_library_flags():
    try:
        pbuild.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not available")
    base = [f for f in pbuild.HIP_FLAGS if f not in ("-Xclang", "-target-feature", "-packed-fp32-ops")]
    assert "-packed-fp32-ops" in pbuild.HIP_FLAGS
    plain = _device_asm(base)
    ours = _device_asm(pbuild.HIP_FLAGS)
    pk = re.compile(r"\bv_pk_(fma|mul|add)_f32\b")
    # the kernel does produce packed FP32 without the flag, so the check is live
    assert pk.search(plain), "control build made no packed FP32 instruction"
    assert not pk.search(ours)
