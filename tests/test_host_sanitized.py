"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(no GPU): pimd_workspace_bytes over the workloads' shapes (parameter checks,
layouts, atom ordering, topology handling, the cell grid and list capacity),
and the ABI checks that run without a device.  The device code is built as
usual; a child process loads the host-sanitized build with clang's shared ASan
runtime (which carries the UBSan handlers) preloaded."""
import glob
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

CHILD = r"""
import ctypes as C
import sys
sys.path.insert(0, %(root)r)
sys.path.insert(0, %(tests)r)
import numpy as np
from paper_2602_13553_amd import build, inputs, pimd
with open("/proc/self/maps") as f:
    assert "libclang_rt.asan" in f.read(), "the ASan runtime is not loaded"
pimd.LIB_PATH = build.LIB_HOST_SAN
lib = pimd.load()
specs = [inputs.harmonic_tiny(), inputs.harmonic_tiny(n_atoms=37, n_beads=3),
         inputs.free_ring_polymer(), inputs.lj_liquid(n_atoms=256, n_beads=8),
         inputs.lj_liquid(n_atoms=171, n_beads=7), inputs.lj_liquid(n_atoms=64, n_beads=32),
         inputs.lj_liquid(n_atoms=4000, n_beads=32), inputs.water(n_atoms=384, n_beads=8),
         inputs.water(n_atoms=99, n_beads=5), inputs.water(n_atoms=32768, n_beads=64),
         inputs.trapped_bosons(), inputs.lj_bosons()]
npt = inputs.lj_liquid(n_atoms=256, n_beads=8)
npt.ensemble, npt.p_ext, npt.tau_p, npt.integrator = inputs.NPT, 0.5, 0.5, 1
aniso = inputs.lj_liquid(n_atoms=256, n_beads=6)
aniso.ensemble, aniso.p_ext, aniso.tau_p, aniso.baro_aniso = inputs.NPH, 0.5, 0.5, 1
specs += [npt, aniso]
for spec in specs:
    for flags in (0, pimd.PIMD_FLAG_VALU_TRANSFORMS, pimd.PIMD_FLAG_CLUSTER_PAIRS):
        p = pimd.params_from_spec(spec, flags)
        keep = []
        t = pimd._topology(spec.lj_active, spec.bonds, keep)
        n = C.c_size_t()
        rc = lib.pimd_workspace_bytes(C.byref(p), pimd._dp(np.ascontiguousarray(spec.mass)),
                                      C.byref(t) if t is not None else None, C.byref(n))
        if flags == pimd.PIMD_FLAG_CLUSTER_PAIRS and rc == pimd.PIMD_ERR_UNSUPPORTED:
            continue   # cluster lists need pair forces without a barostat or bosons
        assert rc == 0 and n.value > 0, (spec.name, flags, rc)
import test_abi
for name in ("test_create_rejects_bad_parameters_without_gpu",
             "test_external_potential_is_accepted_without_gpu",
             "test_flags_are_validated_without_gpu"):
    getattr(test_abi, name)()
print("host-sanitized checks passed")
"""


def _asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_host_code_under_asan_and_ubsan():
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("clang's shared ASan runtime is not installed")
    from paper_2602_13553_amd import build
    build.build(host_sanitize=True)
    env = dict(os.environ)
    env["LD_PRELOAD"] = rt
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([sys.executable, "-c", CHILD % {"root": ROOT, "tests": HERE}],
                       env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "host-sanitized checks passed" in r.stdout
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
