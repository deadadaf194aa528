"""Host logic of the launch-shape autotuner (no GPU): the choice rules and the
header it writes, and the committed table's shape and limits."""
import os
import re

from paper_2602_13553_amd import autotune

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def synthetic_result(pair_time, fused_time, water_pair_time=None):
    rows = []
    for pot, pt in (("lj", pair_time), ("water", water_pair_time)):
        if pt is None:
            continue
        for P in autotune.BEADS:
            for N in autotune.ATOMS:
                rec = {"P": P, "N": N}
                if pot == "water":
                    rec["potential"] = "water"
                elif P in autotune.MFMA_BEADS:
                    rec["fused_mfma"], rec["fused_valu"] = fused_time(P, N)
                for S in autotune.SUBGROUPS:
                    if S * P <= 256:
                        rec["pair_S%d" % S] = pt(P, N, S)
                rows.append(rec)
    return {"device": "test", "steps": 40, "warmup": 10, "rows": rows}


def test_mfma_threshold_is_the_first_size_from_which_mfma_never_loses():
    def fused(P, N):
        # MFMA wins from N = 4096 on, except a dip at N = 8192 for P = 64
        valu = 1e-3 * N
        mfma = valu * (0.9 if N >= 4096 else 1.5)
        if P == 64 and N == 8192:
            mfma = valu * 1.1
        return mfma, valu
    m, _, _ = autotune.choose(synthetic_result(lambda P, N, S: 1.0, fused))
    assert m == [4096 * 16, 4096 * 32, 16384 * 64]


def test_mfma_never_winning_gives_no_threshold():
    m, _, _ = autotune.choose(synthetic_result(lambda P, N, S: 1.0, lambda P, N: (2.0, 1.0)))
    assert all(v >= 1 << 62 for v in m)


def test_subgroups_prefer_fewest_within_two_percent():
    def pair(P, N, S):
        return {1: 10.0, 2: 9.9, 4: 9.0 if N == 64 else 12.0, 8: 13.0, 16: 14.0}[S]
    _, table, water = autotune.choose(synthetic_result(pair, lambda P, N: (1.0, 1.0)))
    assert water == table      # no water points: the water-shaped system takes the LJ table
    assert len(table) == 4 and all(len(r) == 10 for r in table)
    for r in table:
        assert r[0] == 4          # a clear winner is taken
        assert r[1:] == [1] * 9   # 1% slower than S = 2: a tie, fewer sub-groups win


def test_water_points_give_their_own_table():
    res = synthetic_result(lambda P, N, S: float(S), lambda P, N: (1.0, 1.0),
                           water_pair_time=lambda P, N, S: 1.0 / S)
    _, table, water = autotune.choose(res)
    assert all(r == [1] * 10 for r in table)
    for P, r in zip(autotune.BEADS, water):
        assert r == [max(S for S in autotune.SUBGROUPS if S * P <= 256)] * 10


def test_merge_keeps_both_sweeps_and_the_later_point():
    lj = synthetic_result(lambda P, N, S: float(S), lambda P, N: (1.0, 1.0))
    for x in lj["rows"]:
        x.pop("potential", None)             # rows saved before water was swept
    water = synthetic_result(lambda P, N, S: 1.0, lambda P, N: (1.0, 1.0),
                             water_pair_time=lambda P, N, S: 1.0 / S)
    water["rows"] = [x for x in water["rows"] if x.get("potential") == "water"]
    redo = {"device": "test", "steps": 40, "warmup": 10,
            "rows": [{"potential": "lj", "P": 8, "N": 64, "fused_mfma": 1.0, "fused_valu": 1.0,
                      "pair_S1": 9.0, "pair_S2": 9.0, "pair_S4": 9.0, "pair_S8": 9.0,
                      "pair_S16": 1.0}]}
    res = autotune.merge([lj, water, redo])
    assert len(res["rows"]) == 2 * len(lj["rows"])
    _, table, wt = autotune.choose(res)
    assert table[0][0] == 16 and table[0][1:] == [1] * 9
    assert wt[3] == [4] * 10


def test_header_text_declares_every_table():
    res = synthetic_result(lambda P, N, S: float(S), lambda P, N: (1.0, 2.0),
                           water_pair_time=lambda P, N, S: 1.0 / S)
    m, t, w = autotune.choose(res)
    h = autotune.header_text(res, m, t, w)
    for name in ("kMfmaMinBeadAtoms[3]", "kPairSubgroups[4][10]", "kPairSubgroupsWater[4][10]",
                 "kClusterPairs[4][10]"):
        assert name in h
    assert h.count("{1, 1, 1, 1, 1, 1, 1, 1, 1, 1}") == 4
    assert h.count("{4, 4, 4, 4, 4, 4, 4, 4, 4, 4}") == 1


def committed_table(name):
    src = open(os.path.join(ROOT, "paper_2602_13553_amd", "csrc", "pimd_tuning.h")).read()
    body = re.search(name + r"\[4\]\[10\] = \{(.*?)\};", src, re.S).group(1)
    return [[int(v) for v in r.split(",")] for r in re.findall(r"\{([^{}]*)\}", body)]


def test_committed_tables_are_within_limits():
    for name in ("kPairSubgroups", "kPairSubgroupsWater"):
        rows = committed_table(name)
        assert len(rows) == 4 and all(len(r) == 10 for r in rows)
        for P, r in zip(autotune.BEADS, rows):
            for S in r:
                assert S in autotune.SUBGROUPS and S * P <= 256


def test_write_needs_both_workloads(tmp_path, monkeypatch):
    """--write from an LJ-only sweep would replace the water table with the
    LJ one: it refuses, and the header is left alone."""
    import json
    import pytest
    res = synthetic_result(lambda P, N, S: float(S), lambda P, N: (1.0, 1.0))
    path = tmp_path / "lj.json"
    path.write_text(json.dumps(res))
    header = tmp_path / "pimd_tuning.h"
    header.write_text("untouched")
    monkeypatch.setattr(autotune, "HEADER", str(header))
    with pytest.raises(SystemExit):
        autotune.main(["--from-json", str(path), "--write"])
    assert header.read_text() == "untouched"
    water = synthetic_result(lambda P, N, S: 1.0, lambda P, N: (1.0, 1.0),
                             water_pair_time=lambda P, N, S: 1.0 / S)
    water["rows"] = [x for x in water["rows"] if x.get("potential") == "water"]
    wpath = tmp_path / "water.json"
    wpath.write_text(json.dumps(water))
    autotune.main(["--from-json", str(path), "--from-json", str(wpath), "--write"])
    assert "kPairSubgroupsWater[4][10]" in header.read_text()
