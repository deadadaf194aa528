"""Batched execution: every system in a batch evolves exactly as it does alone
(same kernels per system, same noise stream), under step budgets and while
other systems join and leave."""
import numpy as np
import pytest

from paper_2602_13553_amd import inputs

pytestmark = pytest.mark.gpu


def _pimd():
    from paper_2602_13553_amd import pimd
    return pimd


def mixed_specs():
    return [
        inputs.harmonic_tiny(n_atoms=40, n_beads=4, seed=1),            # in-kernel trap, VALU
        inputs.lj_liquid(n_atoms=108, n_beads=8, seed=2),                # VALU transforms
        inputs.lj_liquid(n_atoms=256, n_beads=16, seed=3),               # MFMA P=16
        inputs.lj_liquid(n_atoms=64, n_beads=32, seed=4),                # MFMA P=32, image sums
        inputs.water(n_atoms=192, n_beads=8, seed=5),                    # bonds + masked LJ
        inputs.lj_liquid(n_atoms=171, n_beads=6, seed=6),                # ragged P
        inputs.harmonic_tiny(n_atoms=20, n_beads=64, seed=7),            # MFMA P=64 trap
        inputs.lj_liquid(n_atoms=108, n_beads=5, seed=8),                # odd P: one bead per lane
    ]


def solo(spec, n):
    pimd = _pimd()
    c = pimd.Context.from_spec(spec)
    c.set_state(spec.x0, spec.v0, 0)
    c.step(n)
    out = c.get_state(), c.estimators()
    c.close()
    return out


def test_batch_equals_solo():
    pimd = _pimd()
    specs = mixed_specs()
    b = pimd.Batch()
    ids = [b.add(s) for s in specs]
    for i, s in zip(ids, specs):
        b.set_state(i, s.x0, s.v0, 0)
    b.step(20)
    b.step(3)
    for i, s in zip(ids, specs):
        print("batch vs solo", s.name, flush=True)
        (xs, ps, ss), es = solo(s, 23)
        xb, pb, sb = b.get_state(i)
        eb = b.estimators(i)
        assert sb == ss == 23
        assert np.array_equal(xb, xs), s.name
        assert np.array_equal(pb, ps), s.name
        for n in ("ekin", "espring", "epot", "kcv", "kprim"):
            assert abs(eb[n] - es[n]) <= 1e-12 * max(abs(es["ekin"]), abs(es["espring"])), (s.name, n)
        assert eb["count"] == es["count"] == 23
    b.close()


def test_batch_mixed_splittings_equal_solo():
    """BAOAB and OBABO systems in one batch, on both transform variants (the
    matrix-core groups split by splitting): each equals its solo run."""
    pimd = _pimd()
    M = pimd.PIMD_FLAG_MFMA_TRANSFORMS
    cases = []
    for k, (spec, fl) in enumerate([
            (inputs.harmonic_tiny(n_atoms=40, n_beads=4, seed=11), 0),
            (inputs.lj_liquid(n_atoms=108, n_beads=8, seed=12), 0),
            (inputs.lj_liquid(n_atoms=64, n_beads=32, seed=13), M),
            (inputs.lj_liquid(n_atoms=64, n_beads=32, seed=14), M),
            (inputs.harmonic_tiny(n_atoms=20, n_beads=64, seed=15), M),
            (inputs.water(n_atoms=192, n_beads=16, seed=16), M)]):
        if k % 2 == 1 or k == 4:
            spec.integrator = pimd.PIMD_OBABO
        cases.append((spec, fl))
    b = pimd.Batch()
    ids = [b.add(s, fl) for s, fl in cases]
    for i, (s, fl) in zip(ids, cases):
        b.set_state(i, s.x0, s.v0, 0)
    b.step(12)
    for i, (s, fl) in zip(ids, cases):
        print("batch vs solo", s.name, "obabo" if s.integrator else "baoab", fl, flush=True)
        c = pimd.Context.from_spec(s, flags=fl)
        c.set_state(s.x0, s.v0, 0)
        c.step(12)
        xs, ps, ss = c.get_state()
        c.close()
        xb, pb, sb = b.get_state(i)
        assert sb == ss == 12
        assert np.array_equal(xb, xs), s.name
        assert np.array_equal(pb, ps), s.name
    b.close()


def test_batch_equals_solo_cluster_pairs():
    """Systems whose force pass runs on cluster lists (one falling back to
    per-atom lists in its small box) next to systems on per-atom lists."""
    pimd = _pimd()
    specs = [inputs.lj_liquid(n_atoms=2048, n_beads=32, seed=41),
             inputs.lj_liquid(n_atoms=256, n_beads=8, seed=42),
             inputs.water(n_atoms=1536, n_beads=16, seed=43),
             inputs.lj_liquid(n_atoms=500, n_beads=16, seed=44)]
    flags = [pimd.PIMD_FLAG_CLUSTER_PAIRS] * 3 + [pimd.PIMD_FLAG_ATOM_PAIRS]
    b = pimd.Batch()
    ids = [b.add(s, flags=f) for s, f in zip(specs, flags)]
    for i, s in zip(ids, specs):
        b.set_state(i, s.x0, s.v0, 0)
    b.step(25)
    for i, s, f in zip(ids, specs, flags):
        print("batch vs solo", s.name, f, flush=True)
        c = pimd.Context.from_spec(s, flags=f)
        c.set_state(s.x0, s.v0, 0)
        c.step(25)
        xs, ps, ss = c.get_state()
        c.close()
        xb, pb, sb = b.get_state(i)
        assert sb == ss == 25
        assert np.array_equal(xb, xs), s.name
        assert np.array_equal(pb, ps), s.name
    b.close()


def test_batch_budgets_and_membership():
    pimd = _pimd()
    specs = mixed_specs()[:4]
    b = pimd.Batch()
    ids = [b.add(s) for s in specs]
    for i, s in zip(ids, specs):
        b.set_state(i, s.x0, s.v0, 0)
    budgets = [5, 13, -1, 0]
    for i, n in zip(ids, budgets):
        b.set_budget(i, n)
    b.step(20)
    for i, s, n in zip(ids, specs, budgets):
        want = 20 if n < 0 else n
        (xs, ps, ss), _ = solo(s, want)
        xb, pb, sb = b.get_state(i)
        assert sb == want, (s.name, sb, want)
        assert np.array_equal(xb, xs) and np.array_equal(pb, ps), s.name
    # membership changes: remove one, add a new one, keep stepping
    b.remove(ids[1])
    extra = inputs.lj_liquid(n_atoms=100, n_beads=16, seed=9)
    j = b.add(extra)
    b.set_state(j, extra.x0, extra.v0, 0)
    b.set_budget(ids[0], -1)
    b.step(7)
    (xs, ps, _), _ = solo(extra, 7)
    xb, pb, sb = b.get_state(j)
    assert sb == 7 and np.array_equal(xb, xs) and np.array_equal(pb, ps)
    x0, p0, s0 = b.get_state(ids[0])
    (xs, ps, _), _ = solo(specs[0], 12)
    assert s0 == 12 and np.array_equal(x0, xs) and np.array_equal(p0, ps)
    b.close()
