"""Long-run statistical parity: estimator averages of the GPU path and of the
oracle agree within their combined statistical error.

A chaotic system (the LJ liquid; the water-shaped system) runs for thousands
of steps on both sides from the same seeded start.  The oracle's thermostat
noise is keyed by another seed, so the two runs are independent samples of
the same ensemble and element-wise agreement is not expected (beyond ~10^2
steps it is not even possible).  The oracle's block means are stored in
tests/golden/longrun_oracle.json by tests/golden/make_longrun.py (which calls
only the oracle; a run takes 10-20 host minutes).  Each side's mean of K_PR,
K_CV, T, P_CV and U over the production steps comes with a standard error from
block averages (blocks long against the estimators' correlation time), and
the two means must agree within 4.5 combined standard errors.  The blocks are
long enough for that error to be honest: over four independent oracle runs of
the LJ case the spread of the means matched the mean block standard error
for every estimator (blocks of 300 steps had underestimated it twofold).  For
scale, a 2% error in the temperature moves T's mean by about 20 standard
errors and K_CV's by about 10."""
import json
import math
import os
import sys

import numpy as np
import pytest

from paper_2602_13553_amd import inputs

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "longrun_oracle.json")
NAMES = ("kprim", "kcv", "temp", "pcv", "epot")
Z_BAR = 4.5


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _golden(name):
    with open(GOLDEN) as fh:
        return json.load(fh)[name]


def _spec(case):
    fn = {"lj": inputs.lj_liquid, "water": inputs.water}[case["kind"]]
    return fn(**case["args"])


def gpu_block_means(spec, n_equil, n_blocks, block):
    from paper_2602_13553_amd import pimd
    ctx = pimd.Context.from_spec(spec)
    ctx.set_state(spec.x0, spec.v0, 0)
    ctx.step(n_equil)
    ctx.estimators()
    out = {n: [] for n in NAMES}
    for _ in range(n_blocks):
        ctx.reset_averages()
        ctx.step(block)
        e = ctx.estimators()
        assert e["count"] == block
        for n in NAMES:
            out[n].append(e["sum"][n] / block)
    ctx.close()
    return {n: np.array(v) for n, v in out.items()}


def compare(g, o):
    for n in NAMES:
        mg, mo = g[n].mean(), o[n].mean()
        se = math.sqrt(g[n].var(ddof=1) / len(g[n]) + o[n].var(ddof=1) / len(o[n]))
        z = abs(mg - mo) / se if se > 0 else 0.0
        _say("  %-5s gpu %.6f  oracle %.6f  se %.2e  z %.2f" % (n, mg, mo, se, z))
        assert z <= Z_BAR, (n, mg, mo, se)


@pytest.mark.parametrize("name", ["lj_n256_p8", "water_n648_p8"])
def test_estimator_averages(name):
    """LJ quantum liquid, N = 256, P = 8, with the LJ workload's physics at
    kT = 1.0 (2000 equilibration steps, 8 blocks of 1500); water-shaped
    system, 216 molecules, P = 8, 300 K, dt = 0.25 fs (2000 equilibration
    steps, 8 blocks of 1000).  The GPU side runs with the seed of the input
    spec, the oracle's stored run with that seed + 7777."""
    case = _golden(name)
    spec = _spec(case)
    assert case["oracle_seed"] != spec.seed
    _say("case %s equil=%d blocks=%dx%d" % (name, case["n_equil"], case["n_blocks"],
                                            case["block"]))
    g = gpu_block_means(spec, case["n_equil"], case["n_blocks"], case["block"])
    o = {n: np.array(case["block_means"][n]) for n in NAMES}
    compare(g, o)
