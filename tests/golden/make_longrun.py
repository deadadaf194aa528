"""Writes tests/golden/longrun_oracle.json: the oracle's block averages of the
estimators (App. A: K_PR, K_CV, T, P_CV, U) over long runs of two chaotic
systems, for the GPU's long-run statistical parity test.

Calls only the oracle and the seeded input generators.  The oracle's
thermostat noise is keyed by a seed other than the GPU run's, so the two runs
are independent samples of the same ensemble.  A run takes 10-20 minutes of
host time (the oracle's forces are all-pairs); the GPU test reads the stored
means instead of repeating it.

    python tests/golden/make_longrun.py [case ...]
"""
from __future__ import annotations

import copy
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2602_13553_amd import inputs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "longrun_oracle.json")
NAMES = ("kprim", "kcv", "temp", "pcv", "epot")
ORACLE_SEED_OFFSET = 7777

# LJ quantum liquid with the LJ workload's physics (hbar = 0.1, dt = 0.002,
# tau = 0.5, rho = 0.8) at kT = 1.0, where the FCC start melts within the
# equilibration; water-shaped system of 216 molecules (box 18.6 A > 2 rc) at
# 300 K, dt = 0.25 fs.
CASES = {
    "lj_n256_p8": dict(kind="lj", args=dict(n_atoms=256, n_beads=8, seed=11, kT=1.0),
                       n_equil=2000, n_blocks=8, block=1500),
    "water_n648_p8": dict(kind="water", args=dict(n_atoms=648, n_beads=8, seed=3),
                          n_equil=2000, n_blocks=8, block=1000),
}


def make_spec(case):
    fn = {"lj": inputs.lj_liquid, "water": inputs.water}[case["kind"]]
    return fn(**case["args"])


def oracle_block_means(spec, n_equil, n_blocks, block):
    st = oracle.State.from_spec(spec)
    st.step(n_equil)
    out = {n: [] for n in NAMES}
    for _ in range(n_blocks):
        acc = {n: 0.0 for n in NAMES}
        for _ in range(block):
            st.step(1)
            e = st.estimators()
            for n in NAMES:
                acc[n] += e[n]
        for n in NAMES:
            out[n].append(acc[n] / block)
    return out


def main(names):
    for name in names:
        case = CASES[name]
        spec = make_spec(case)
        ospec = copy.copy(spec)
        ospec.seed = spec.seed + ORACLE_SEED_OFFSET
        t0 = time.time()
        means = oracle_block_means(ospec, case["n_equil"], case["n_blocks"], case["block"])
        print("%s: %.0f s" % (name, time.time() - t0), flush=True)
        data = {}
        if os.path.exists(OUT):
            with open(OUT) as fh:
                data = json.load(fh)
        data[name] = dict(case, oracle_seed=ospec.seed, block_means=means)
        with open(OUT, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(CASES))
