"""Autotuner for libpimd.so's launch shapes, run on the GPU the library targets.

It sweeps two workloads over the grid P in {8, 16, 32, 64} and
N = 64, 128, ..., 32768:

* LJ quantum liquids with the batched workload's physics: reduced density
  0.8, kT 0.7, hbar 0.1, rc 2.5, dt 0.002, tau 0.5;
* the water-shaped system (O-O LJ cut at 9 A plus O-H bonds, 1 g/cm^3,
  300 K), with N rounded up to whole molecules.  Its force items are
  bimodal (an O carries a long O-O list, an H only its bond), so its best
  lane split differs from the liquid's.

For each system it times the following, with HIP events on the library's
stream over the same steps:

* the step pass with matrix-core (MFMA) and with vector-ALU transforms
  (P = 16, 32, 64, LJ only: the step pass does not depend on the potential);
* the force pass with S = 1, 2, 4, 8, 16 lane sub-groups per atom (S*P <= 256).

From the timings it picks three things:

* per P, the smallest N*P from which the matrix cores are at least as fast
  at every larger size of the sweep;
* per (P, N), the fewest sub-groups S within 2% of the fastest, once for
  LJ and once for the water-shaped system.

With --write it rewrites csrc/pimd_tuning.h. The library compiles that table
in, so a given system always gets the same launch shapes. Runs are then
reproducible, and a system in a batch matches its solo run bit for bit.
Rebuild the library (``__graft_entry__.build()``) after writing.

    python -m paper_2602_13553_amd.autotune [--write] [--steps 40] [--json out.json] [--only water]
    python -m paper_2602_13553_amd.autotune --from-json a.json [--from-json b.json] --write   (no GPU)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

from . import inputs, pimd

HERE = os.path.dirname(os.path.abspath(__file__))
HEADER = os.path.join(HERE, "csrc", "pimd_tuning.h")

POTENTIALS = ("lj", "water")
BEADS = (8, 16, 32, 64)
ATOMS = tuple(2 ** k for k in range(6, 16))          # 64 ... 32768
SUBGROUPS = (1, 2, 4, 8, 16)
MFMA_BEADS = (16, 32, 64)


def time_kernels(spec, flags: int, steps: int, warmup: int) -> dict:
    """Average per-launch time (ms) of each kernel kind over `steps` steps."""
    ctx = pimd.Context.from_spec(spec, flags=flags)
    try:
        ctx.set_state(spec.x0, spec.v0, 0)
        ctx.step(warmup)
        ctx.profile_begin()
        ctx.step(steps)
        prof = ctx.profile_end()
    finally:
        ctx.close()
    return {k: (ms / n if n else 0.0) for k, (n, ms) in prof.items()}


def sweep(steps: int = 40, warmup: int = 10, log=print, potentials=POTENTIALS) -> dict:
    rows = []
    for pot in potentials:
        for P in BEADS:
            for N in ATOMS:
                if pot == "lj":
                    spec = inputs.lj_liquid(n_atoms=N, n_beads=P)
                else:
                    spec = inputs.water(n_atoms=3 * -(-N // 3), n_beads=P)
                rec = {"potential": pot, "P": P, "N": N}
                if pot == "lj" and P in MFMA_BEADS:
                    for tag, fl in (("mfma", pimd.PIMD_FLAG_MFMA_TRANSFORMS),
                                    ("valu", pimd.PIMD_FLAG_VALU_TRANSFORMS)):
                        rec["fused_" + tag] = time_kernels(spec, fl, steps, warmup)["fused"]
                for S in SUBGROUPS:
                    if S * P > 256:
                        continue
                    rec["pair_S%d" % S] = time_kernels(spec, pimd.PIMD_PAIR_SUBGROUPS(S),
                                                       steps, warmup)["pair"]
                rows.append(rec)
                log(json.dumps(rec))
    return {"device": _device_name(), "steps": steps, "warmup": warmup, "rows": rows}


def merge(results: list) -> dict:
    """One sweep from several saved ones; a later file's point replaces an
    earlier one's.  Rows saved without a potential are LJ rows."""
    out = dict(results[0])
    by_key = {}
    for res in results:
        for x in res["rows"]:
            x = dict(x)
            x.setdefault("potential", "lj")
            by_key[(x["potential"], x["P"], x["N"])] = x
    out["rows"] = list(by_key.values())
    return out


def _device_name() -> str:
    try:
        import torch
        pr = torch.cuda.get_device_properties(0)
        return "%s (%s)" % (pr.name, getattr(pr, "gcnArchName", "?"))
    except Exception:       # the table still records where it came from
        return "unknown"


def _rows(result: dict, pot: str) -> list:
    return [x for x in result["rows"] if x.get("potential", "lj") == pot]


def _subgroup_table(rows: list) -> list:
    table = []
    for P in BEADS:
        line = []
        for N in ATOMS:
            x = next(x for x in rows if x["P"] == P and x["N"] == N)
            cand = {S: x["pair_S%d" % S] for S in SUBGROUPS if "pair_S%d" % S in x}
            # the fewest sub-groups within 2% of the fastest: points closer
            # than that are ties at 40 timed steps
            best = min(cand.values())
            line.append(min(S for S, v in cand.items() if v <= 1.02 * best))
        table.append(line)
    return table


def choose(result: dict) -> tuple[list, list, list]:
    """(kMfmaMinBeadAtoms, LJ sub-group table, water sub-group table).  A
    sweep without water points gives the water-shaped system the LJ table."""
    rows = _rows(result, "lj")
    mfma_min = []
    for P in MFMA_BEADS:
        r = sorted((x for x in rows if x["P"] == P), key=lambda x: x["N"])
        thr = None
        # the smallest size from which MFMA is never slower (2% grace)
        for i in range(len(r)):
            if all(x["fused_mfma"] <= 1.02 * x["fused_valu"] for x in r[i:]):
                thr = r[i]["N"] * P
                break
        mfma_min.append(thr if thr is not None else 1 << 62)
    table = _subgroup_table(rows)
    water = _rows(result, "water")
    return mfma_min, table, (_subgroup_table(water) if water else table)


def _c_rows(table: list) -> str:
    return ",\n".join("    {" + ", ".join(str(v) for v in line) + "}" for line in table)


def header_text(result: dict, mfma_min: list, table: list, water: list) -> str:
    stamp = time.strftime("%Y-%m-%d")
    return (
        "// Launch-shape table of libpimd.so.  Written by paper_2602_13553_amd/autotune.py\n"
        "// from kernel timings on the GPU; regenerate with\n"
        "//   python -m paper_2602_13553_amd.autotune --write\n"
        "// (the sweep, its workloads and the raw timings are described there).\n"
        "// Measured on %s, %s, %d timed steps per point.\n"
        "#pragma once\n\n"
        "namespace pimd {\n"
        "namespace tuning {\n\n"
        "// Smallest N*P from which the matrix-core step pass is faster than the\n"
        "// vector-ALU one, for P = 16, 32, 64.\n"
        "constexpr long long kMfmaMinBeadAtoms[3] = {%s};\n\n"
        "// Force-pass lane sub-groups per atom for P = 8, 16, 32, 64 (rows) and N in\n"
        "// [2^6, 2^7), [2^7, 2^8), ..., [2^15, 2^16) (columns; clamped at both ends),\n"
        "// for LJ liquids.  0: the occupancy heuristic decides.\n"
        "constexpr int kPairSubgroups[4][10] = {\n%s,\n};\n\n"
        "// The same for the water-shaped potential (O-O LJ plus O-H bonds).\n"
        "constexpr int kPairSubgroupsWater[4][10] = {\n%s,\n};\n\n"
        "// Force pass on cluster lists (1) or per-atom lists (0), same rows and\n"
        "// columns as kPairSubgroups.  The sweep does not time cluster lists (they\n"
        "// were slower than per-atom lists at every size measured), so they stay off.\n"
        "constexpr int kClusterPairs[4][10] = {\n%s,\n};\n\n"
        "}  // namespace tuning\n"
        "}  // namespace pimd\n"
        % (result["device"], stamp, result["steps"],
           ", ".join("%dLL" % v for v in mfma_min), _c_rows(table), _c_rows(water),
           ",\n".join("    {" + ", ".join("0" for _ in line) + "}" for line in table)))


def summary_text(result: dict, mfma_min: list, table: list, water: list) -> str:
    out = ["# fused pass (us): matrix cores vs vector ALUs; force pass (us) per S",
           "%-6s %4s %6s %10s %10s  %s" % ("pot", "P", "N", "mfma", "valu", "pair S=1,2,4,8,16")]
    for pot in POTENTIALS:
        for x in _rows(result, pot):
            pr = " ".join("%8.2f" % (1e3 * x["pair_S%d" % S]) if "pair_S%d" % S in x else "%8s" % "-"
                          for S in SUBGROUPS)
            out.append("%-6s %4d %6d %10s %10s  %s" % (
                pot, x["P"], x["N"],
                "%.2f" % (1e3 * x["fused_mfma"]) if "fused_mfma" in x else "-",
                "%.2f" % (1e3 * x["fused_valu"]) if "fused_valu" in x else "-", pr))
    out.append("kMfmaMinBeadAtoms (P=16,32,64): %s" % mfma_min)
    out.append("kPairSubgroups (rows P=8,16,32,64; cols N=2^6..2^15): %s" % table)
    out.append("kPairSubgroupsWater (same rows and cols): %s" % water)
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--write", action="store_true", help="rewrite csrc/pimd_tuning.h")
    ap.add_argument("--json", help="also save the raw timings here")
    ap.add_argument("--from-json", action="append",
                    help="take the timings from saved sweeps instead of the GPU (repeatable)")
    ap.add_argument("--only", choices=POTENTIALS, help="sweep one workload only")
    args = ap.parse_args(argv)
    if args.from_json:
        saved = []
        for path in args.from_json:
            with open(path) as f:
                saved.append(json.load(f))
        res = merge(saved)
    else:
        res = sweep(args.steps, args.warmup, log=lambda m: print(m, file=sys.stderr, flush=True),
                    potentials=(args.only,) if args.only else POTENTIALS)
    if args.json:
        with open(args.json, "w") as f:
            json.dump(res, f, indent=1)
    if not _rows(res, "lj"):
        # a water-only sweep: merge it with an LJ one (--from-json twice) to
        # pick the tables
        print("no LJ points: saved the timings only", flush=True)
        return
    mfma_min, table, water = choose(res)
    print(summary_text(res, mfma_min, table, water), flush=True)
    if args.write and not _rows(res, "water"):
        # the header would give the water-shaped potential the LJ table
        sys.exit("no water points: not writing %s (merge a water sweep with --from-json)" % HEADER)
    if args.write:
        with open(HEADER, "w") as f:
            f.write(header_text(res, mfma_min, table, water))
        print("wrote %s" % HEADER, flush=True)


if __name__ == "__main__":
    main()
