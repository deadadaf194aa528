"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: its C
code built with both (every finding fatal) and the pins run against that
build in a child process with the sanitizer runtimes preloaded.  An
out-of-bounds access, use after free, signed overflow, misaligned access or
other undefined behaviour anywhere the pins reach fails this test."""
import os
import subprocess
import sys

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

# every pin except the long statistical runs (a few minutes under the
# sanitizers), which exercise the same code as the short ones
SUBSET = ("not (harmonic_config_x2 or mode_variances or bzp_barostat_equipartition or "
          "bzp_barostat_thermostat_rate or thermostat_equipartition or exact_trap_energy)")


def _runtime(name):
    out = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True)
    path = out.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_pins_under_asan_and_ubsan():
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc's sanitizer runtimes are not installed")
    lib = oracle.build(force=True, sanitize=True)
    env = dict(os.environ)
    env["ORACLE_LIB"] = lib
    env["LD_PRELOAD"] = asan + ":" + ubsan
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["OMP_NUM_THREADS"] = "4"
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(HERE, "test_oracle_pins.py"),
                        "-q", "-x", "-p", "no:cacheprovider", "-k", SUBSET],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=1500)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
    assert " passed" in r.stdout, tail
