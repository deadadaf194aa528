"""GPU parity: the HIP path (through the C ABI) against the CPU oracle,
element by element on identical seeded inputs and noise streams.

Bar: max|a_gpu - a_orc| <= 1e-12 * max|a_orc| for positions and momenta
(after 10 steps for the chaotic pair potentials; over the whole run for the
linear harmonic system).  Estimators: 1e-10 relative to their scale (they are
sums of up to ~1e8 terms with cancellation in K_CV)."""
import math
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2602_13553_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _pimd():
    from paper_2602_13553_amd import pimd
    return pimd


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_err(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def run_pair(spec, nsteps, chunks=None, flags=0):
    """Run the GPU and the oracle from the spec's state; return both states."""
    pimd = _pimd()
    _say("case %s nsteps=%d flags=%d" % (spec.name, nsteps, flags))
    ctx = pimd.Context.from_spec(spec, flags=flags)
    ctx.set_state(spec.x0, spec.v0, 0)
    for c in (chunks or [nsteps]):
        ctx.step(c)
    est = ctx.estimators()
    gx, gp, gs = ctx.get_state()
    ctx.close()
    st = oracle.State.from_spec(spec)
    st.step(nsteps)
    return (gx, gp, gs, est), (st.x, st.p, int(st.step_count[0]), st.estimators(), st.sys)


def pressure_scales(s, x, est):
    """Sizes of the terms of P_CV, P_PR and P_MD for system s at positions x
    [P][N][3]: the bar for each pressure is relative to it, since the terms
    largely cancel.  Zero where the pressures are not defined (no box)."""
    if s.pot != oracle.POT_PAIR or not s.box[0] > 0:
        return {"pcv": 0.0, "ppr": 0.0, "pmd": 0.0}
    P, N = x.shape[0], x.shape[1]
    f, _ = s.forces(x)
    vir = np.abs((x - x.mean(axis=0)) * f).sum()
    w = sum(abs(s.virial(x[k])) for k in range(P))
    v3 = 3 * float(np.prod(s.box))
    ek, es = abs(est["ekin"]), abs(est["espring"])
    return {"pcv": (2 * ek + vir + w) / (P * v3),
            "ppr": (3 * P * N * s.kB * s.temp + (2 * es + w) / P) / v3,
            "pmd": (2 * ek + w) / v3}


def check_states(g, o, tol=TOL, est_tol=1e-10):
    gx, gp, gs, gest = g
    ox, op, os_, oest, osys = o
    assert gs == os_
    ex, ep = rel_err(gx, ox), rel_err(gp, op)
    _say("  x rel %.3e  p rel %.3e" % (ex, ep))
    assert ex <= tol, ex
    assert ep <= tol, ep
    scale = max(abs(oest["ekin"]), abs(oest["espring"]), abs(oest["epot"]), 1e-300)
    for name in ("ekin", "espring", "epot", "etot", "kprim", "kcv"):
        assert abs(gest[name] - oest[name]) <= est_tol * scale, (name, gest[name], oest[name])
    assert abs(gest["temp"] - oest["temp"]) <= est_tol * abs(oest["temp"])
    for name, psc in pressure_scales(osys, ox, oest).items():
        _say("  %s %.10e (oracle %.10e, scale %.3e)" % (name, gest[name], oest[name], psc))
        assert abs(gest[name] - oest[name]) <= est_tol * psc, (name, gest[name], oest[name])


# ------------------------------------------------------------ harmonic trap
def test_harmonic_config_full_run():
    """N=64, P=4, kT=0.25, 2000 steps: linear and contracting, so parity holds
    over the whole run."""
    spec = inputs.harmonic_tiny()
    g, o = run_pair(spec, 2000)
    check_states(g, o)


@pytest.mark.parametrize("N,P", [(1, 1), (37, 3), (50, 5), (33, 7), (19, 16), (5, 64), (3, 128)])
def test_harmonic_ragged_and_odd(N, P):
    spec = inputs.harmonic_tiny(n_atoms=N, n_beads=P, seed=100 + N + P)
    g, o = run_pair(spec, 40, chunks=[1, 7, 32])
    check_states(g, o)


def test_max_beads_large_system_sampled():
    """P = 128 (the largest the library takes) on 2^19 trapped atoms: 2^26
    bead*atoms, 1.6 GB per state array, grids far past one wave of blocks.
    The atoms of a trap do not interact, so the oracle steps a sample of them
    alone, with their own indices in the noise counter, and the GPU's
    positions and momenta of those atoms must match element by element."""
    pimd = _pimd()
    N, P, nsteps = 1 << 19, 128, 2
    spec = inputs.harmonic_tiny(n_atoms=N, n_beads=P, seed=5)
    _say("case harmonic N=%d P=%d nsteps=%d" % (N, P, nsteps))
    ctx = pimd.Context.from_spec(spec)
    ctx.set_state(spec.x0, spec.v0, 0)
    ctx.step(nsteps)
    est = ctx.estimators()
    gx, gp, gs = ctx.get_state()
    ctx.close()
    assert gs == nsteps and est["nonfinite"] == 0
    idx = np.sort(np.random.default_rng(1).choice(N, 48, replace=False))
    idx = np.concatenate([[0, 1], idx, [N - 2, N - 1]])
    sub = oracle.System.from_spec(spec)
    sub.n_atoms, sub.mass, sub.atom_id = len(idx), np.asarray(spec.mass)[idx], idx
    st = oracle.State(sub, spec.x0[:, idx], spec.v0[:, idx])
    st.step(nsteps)
    ex, ep = rel_err(gx[:, idx], st.x), rel_err(gp[:, idx], st.p)
    _say("  sampled x rel %.3e  p rel %.3e" % (ex, ep))
    assert ex <= TOL and ep <= TOL


def test_free_ring_polymer_nve():
    spec = inputs.free_ring_polymer(n_atoms=29, n_beads=8, dt=0.05)
    g, o = run_pair(spec, 200)
    check_states(g, o)


def test_harmonic_nve():
    spec = inputs.harmonic_tiny(n_atoms=20, n_beads=6, ensemble=inputs.NVE)
    g, o = run_pair(spec, 300)
    check_states(g, o)


# ------------------------------------------------------------ Lennard-Jones
def test_lj_small():
    spec = inputs.lj_liquid(n_atoms=256, n_beads=8, seed=11)
    g, o = run_pair(spec, 10)
    check_states(g, o)


@pytest.mark.parametrize("N,P", [(64, 16), (100, 8), (30, 4)])
def test_lj_small_box_images(N, P):
    """Boxes with L < 2 rc: the force is the sum over periodic images."""
    spec = inputs.lj_liquid(n_atoms=N, n_beads=P, seed=N)
    assert spec.box[0] < 2 * spec.lj_rc
    g, o = run_pair(spec, 10)
    check_states(g, o)


def test_lj_ragged_beads():
    spec = inputs.lj_liquid(n_atoms=171, n_beads=6, seed=5)
    g, o = run_pair(spec, 10, chunks=[3, 7])
    check_states(g, o)


def test_lj_full_size():
    """N=4000, P=32 (the LJ quantum-liquid workload), 10 steps."""
    spec = inputs.lj_liquid()
    g, o = run_pair(spec, 10)
    check_states(g, o)


# ------------------------------------------------------------ water-shaped
def test_water_small():
    spec = inputs.water(n_atoms=384, n_beads=8, seed=3)
    g, o = run_pair(spec, 10)
    check_states(g, o)


def test_water_full_size_p32():
    """N=32766 (10922 molecules), P=32, 10 steps."""
    spec = inputs.water(n_beads=32)
    g, o = run_pair(spec, 10)
    check_states(g, o)


def test_water_full_size_p64():
    """N=32766, P=64 (the largest water-shaped workload), 10 steps."""
    spec = inputs.water(n_beads=64)
    g, o = run_pair(spec, 10)
    check_states(g, o)


@pytest.mark.parametrize("kind,N,P", [("lj", 257, 64), ("lj_images", 64, 64), ("water", 387, 64),
                                      ("lj", 130, 128)])
def test_pair_one_group_per_atom(kind, N, P):
    """The force pass with one lane group per atom (S = 1) at P = 64 and 128:
    the lanes take bead pairs, in two sub-groups per atom of half a wave
    (P = 64) or a whole wave (P = 128), with 16-byte gathers and the image
    shift applied only where it is not zero.  A ragged last tile, a box under
    2 rc (every pair through images, entries with several shifts), water's
    bonds."""
    pimd = _pimd()
    if kind == "water":
        spec = inputs.water(n_atoms=N, n_beads=P, seed=N)
    else:
        spec = inputs.lj_liquid(n_atoms=N, n_beads=P, seed=N)
        if kind == "lj_images":
            assert spec.box[0] < 2 * spec.lj_rc
    g, o = run_pair(spec, 6, chunks=[2, 4], flags=pimd.PIMD_PAIR_SUBGROUPS(1))
    check_states(g, o)


def _tuning_table(name):
    import re
    src = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                            "paper_2602_13553_amd", "csrc", "pimd_tuning.h")).read()
    body = re.search(name + r"\[4\]\[10\] = \{(.*?)\};", src, re.S).group(1)
    return [[int(v) for v in r.split(",")] for r in re.findall(r"\{([^{}]*)\}", body)]


def test_pair_subgroups_follow_the_tuning_table_of_the_potential():
    """With no sub-group flag, the force pass takes its lane split from the
    compiled table of its potential, indexed by P and floor(log2 N)."""
    pimd = _pimd()
    tables = {"lj": _tuning_table("kPairSubgroups"), "water": _tuning_table("kPairSubgroupsWater")}
    for kind, N, P in (("water", 32766, 32), ("water", 32766, 64), ("water", 2049, 8),
                       ("water", 300, 16), ("lj", 4000, 32), ("lj", 300, 16)):
        spec = (inputs.water(n_atoms=N, n_beads=P) if kind == "water"
                else inputs.lj_liquid(n_atoms=N, n_beads=P))
        col = min(max(spec.n_atoms.bit_length() - 1 - 6, 0), 9)
        want = tables[kind][(8, 16, 32, 64).index(P)][col]
        ctx = pimd.Context.from_spec(spec)
        info = ctx.launch_info()
        ctx.close()
        assert info["pair_subgroups"] == want, (kind, N, P)


@pytest.mark.parametrize("kind,N,P,S", [("lj", 257, 32, 4), ("lj", 130, 16, 8), ("water", 387, 8, 2),
                                        ("lj", 60, 4, 16), ("lj", 50, 2, 16),
                                        ("lj", 131, 7, 4), ("lj", 100, 33, 2), ("water", 99, 5, 1)])
def test_pair_lane_layouts(kind, N, P, S):
    """Both lane layouts of the force pass at several sub-group counts: bead
    pairs for even P (2S sub-groups of P/2 lanes, summed per bead in
    sub-group order) and one bead per lane for odd P, with ragged last tiles
    and water's bonds; the context reports which one it runs."""
    pimd = _pimd()
    if kind == "water":
        spec = inputs.water(n_atoms=N, n_beads=P, seed=N)
    else:
        spec = inputs.lj_liquid(n_atoms=N, n_beads=P, seed=N)
    flags = pimd.PIMD_PAIR_SUBGROUPS(S)
    ctx = pimd.Context.from_spec(spec, flags=flags)
    info = ctx.launch_info()
    ctx.close()
    assert info["pair_subgroups"] == S
    assert info["bead_pairs"] == (1 if P % 2 == 0 else 0)
    g, o = run_pair(spec, 6, chunks=[2, 4], flags=flags)
    check_states(g, o)


# ------------------------------------------------------------ transform variants
@pytest.mark.parametrize("kind,N,P", [
    ("harmonic", 37, 16), ("harmonic", 50, 32), ("harmonic", 5, 64), ("harmonic", 333, 64),
    ("lj", 250, 16), ("lj", 500, 32), ("lj", 130, 64), ("water", 387, 32), ("water", 99, 64)])
def test_mfma_transforms(kind, N, P):
    """The matrix-core step pass forced on small systems: ragged last tiles
    (N not a multiple of the 16-atom tile or of the block tile), the trap path
    and the pair path, for each bead count it supports."""
    pimd = _pimd()
    fl = pimd.PIMD_FLAG_MFMA_TRANSFORMS
    if kind == "harmonic":
        spec = inputs.harmonic_tiny(n_atoms=N, n_beads=P, seed=7 * N + P)
        g, o = run_pair(spec, 40, chunks=[1, 7, 32], flags=fl)
    elif kind == "lj":
        spec = inputs.lj_liquid(n_atoms=N, n_beads=P, seed=N + P)
        g, o = run_pair(spec, 10, chunks=[4, 6], flags=fl)
    else:
        spec = inputs.water(n_atoms=N, n_beads=P, seed=N)
        g, o = run_pair(spec, 10, flags=fl)
    check_states(g, o)


def test_valu_transforms_water_full_size():
    """The vector-ALU step pass at the water-shaped workload's size (the size
    picks the matrix cores by default)."""
    pimd = _pimd()
    spec = inputs.water(n_beads=32)
    g, o = run_pair(spec, 5, flags=pimd.PIMD_FLAG_VALU_TRANSFORMS)
    check_states(g, o)


# ------------------------------------------------------------ OBABO splitting
@pytest.mark.parametrize("kind,N,P,mfma", [
    ("harmonic", 37, 8, False), ("harmonic", 50, 32, True), ("lj", 256, 8, False),
    ("lj", 130, 64, True), ("water", 387, 32, False), ("water", 99, 16, True)])
def test_obabo_matches_oracle(kind, N, P, mfma):
    """O(dt/2) B A(dt) B O(dt/2), the two O steps with their own draws, on the
    trap (in-kernel forces) and the pair potentials (the closing pass carries
    the second O), on both transform variants."""
    pimd = _pimd()
    if kind == "harmonic":
        spec = inputs.harmonic_tiny(n_atoms=N, n_beads=P, seed=3 * N + P)
    elif kind == "lj":
        spec = inputs.lj_liquid(n_atoms=N, n_beads=P, seed=N + 2 * P)
    else:
        spec = inputs.water(n_atoms=N, n_beads=P, seed=N + 1)
    spec.integrator = pimd.PIMD_OBABO
    g, o = run_pair(spec, 10, chunks=[1, 7, 2],
                    flags=pimd.PIMD_FLAG_MFMA_TRANSFORMS if mfma else 0)
    check_states(g, o)


# ------------------------------------------------------------ fixcom
@pytest.mark.parametrize("kind,N,P,mfma,obabo", [
    ("harmonic", 37, 8, False, False), ("harmonic", 50, 32, True, False),
    ("lj", 256, 8, False, False), ("lj", 130, 64, True, False), ("water", 387, 32, False, False),
    ("lj", 108, 8, False, True), ("harmonic", 20, 16, True, True)])
def test_fixcom_matches_oracle(kind, N, P, mfma, obabo):
    """The centroids' center-of-mass velocity removed at the end of every step:
    in-kernel for the trap, through a closing pass of its own before each step
    with the pair potentials; estimators of the state after the removal."""
    pimd = _pimd()
    if kind == "harmonic":
        spec = inputs.harmonic_tiny(n_atoms=N, n_beads=P, seed=5 * N + P)
    elif kind == "lj":
        spec = inputs.lj_liquid(n_atoms=N, n_beads=P, seed=N + 3 * P)
    else:
        spec = inputs.water(n_atoms=N, n_beads=P, seed=N + 2)
    spec.fixcom = 1
    spec.integrator = pimd.PIMD_OBABO if obabo else pimd.PIMD_BAOAB
    g, o = run_pair(spec, 10, chunks=[1, 7, 2],
                    flags=pimd.PIMD_FLAG_MFMA_TRANSFORMS if mfma else 0)
    check_states(g, o)
    gx, gp, gs, gest = g
    mass = np.asarray(spec.mass)
    com = (gp.mean(axis=0)).sum(axis=0) / mass.sum()   # centroid COM velocity
    assert np.abs(com).max() <= 1e-12 * np.abs(gp / mass[None, :, None]).max()
    assert gest["count"] == 10


# ------------------------------------------------------------ cluster lists
@pytest.mark.parametrize("case", ["lj_full", "lj_p16", "lj_small_box", "water_p32", "water_small"])
def test_cluster_pairs(case):
    """The force pass on cluster lists (shared neighbor rows staged in LDS),
    forced by flag, against the oracle.  The small boxes exercise the
    per-block fallback to per-atom lists (cluster wider than the box allows);
    the LJ runs span list rebuilds."""
    pimd = _pimd()
    spec, n = {
        "lj_full": (inputs.lj_liquid(), 30),
        "lj_p16": (inputs.lj_liquid(n_atoms=1372, n_beads=16, seed=21), 40),
        "lj_small_box": (inputs.lj_liquid(n_atoms=256, n_beads=8, seed=11), 10),
        "water_p32": (inputs.water(n_beads=32), 10),
        "water_small": (inputs.water(n_atoms=384, n_beads=8, seed=3), 10),
    }[case]
    ctx = pimd.Context.from_spec(spec, flags=pimd.PIMD_FLAG_CLUSTER_PAIRS)
    assert ctx.launch_info()["cluster_pairs"] == 1
    ctx.close()
    g, o = run_pair(spec, n, flags=pimd.PIMD_FLAG_CLUSTER_PAIRS)
    check_states(g, o)
    _say("  rebuilds %d" % g[3]["n_rebuilds"])


def test_cluster_pairs_match_atom_pairs():
    """The same LJ state through both force paths: same trajectory to
    rounding (pair sums in a different order)."""
    pimd = _pimd()
    spec = inputs.lj_liquid(n_atoms=2048, n_beads=32, seed=31)
    out = []
    for fl in (pimd.PIMD_FLAG_CLUSTER_PAIRS, pimd.PIMD_FLAG_ATOM_PAIRS):
        ctx = pimd.Context.from_spec(spec, flags=fl)
        ctx.set_state(spec.x0, spec.v0, 0)
        ctx.step(20)
        out.append(ctx.get_state())
        ctx.close()
    assert rel_err(out[0][0], out[1][0]) <= TOL
    assert rel_err(out[0][1], out[1][1]) <= TOL


# ------------------------------------------------------------ running sums
def test_running_sums_match_oracle_per_step():
    spec = inputs.lj_liquid(n_atoms=108, n_beads=8, seed=21)
    pimd = _pimd()
    ctx = pimd.Context.from_spec(spec)
    ctx.set_state(spec.x0, spec.v0, 0)
    ctx.step(6)
    e = ctx.estimators()
    ctx.close()
    st = oracle.State.from_spec(spec)
    acc = {n: [] for n in oracle.ESTIMATOR_NAMES}
    for _ in range(6):
        st.step(1)
        for n, v in st.estimators().items():
            acc[n].append(v)
    assert e["count"] == 6
    psc = pressure_scales(st.sys, st.x, {q: acc[q][-1] for q in acc})
    for n in oracle.ESTIMATOR_NAMES:
        s = sum(acc[n])
        sc = max(abs(x) for x in acc[n] + [psc.get(n, 0.0)]) * 6
        assert abs(e["sum"][n] - s) <= 1e-10 * sc, n
        assert abs(e["sumsq"][n] - sum(x * x for x in acc[n])) <= 1e-10 * sc * sc / 6, n


# ------------------------------------------------------------ determinism, restart, graphs
def test_bitwise_deterministic_and_graph_equivalent():
    spec = inputs.lj_liquid(n_atoms=500, n_beads=16, seed=2)
    pimd = _pimd()
    outs = []
    for chunks in ([64], [64], [32, 32], [1] * 64):
        ctx = pimd.Context.from_spec(spec)
        ctx.set_state(spec.x0, spec.v0, 0)
        for c in chunks:
            ctx.step(c)
        outs.append(ctx.get_state())
        ctx.close()
    for x, p, s in outs[1:]:
        assert np.array_equal(x, outs[0][0]) and np.array_equal(p, outs[0][1]) and s == 64


def test_no_graph_path_with_profiling():
    """PIMD_FLAG_NO_GRAPHS takes the path a context falls back to when graph
    capture fails: every step launched one by one.  Profiling, stepping and
    destroying the context then work, the profile counts every launch, and
    the trajectory equals the graph-replayed one bit for bit."""
    spec = inputs.lj_liquid(n_atoms=500, n_beads=16, seed=2)
    pimd = _pimd()
    outs = []
    for flags in (0, pimd.PIMD_FLAG_NO_GRAPHS):
        ctx = pimd.Context.from_spec(spec, flags=flags)
        ctx.set_state(spec.x0, spec.v0, 0)
        ctx.step(64)
        ctx.profile_begin()
        ctx.step(64)
        prof = ctx.profile_end()
        ctx.step(64)
        outs.append(ctx.get_state())
        ctx.close()
        assert sum(n for n, _ in prof.values()) >= 2 * 64, prof
        assert all(ms >= 0.0 for _, ms in prof.values()), prof
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    assert outs[0][2] == outs[1][2] == 192


def test_checkpoint_restart():
    spec = inputs.lj_liquid(n_atoms=256, n_beads=8, seed=8)
    pimd = _pimd()
    a = pimd.Context.from_spec(spec)
    a.set_state(spec.x0, spec.v0, 0)
    a.step(20)
    xa, pa, sa = a.get_state()
    a.close()
    b = pimd.Context.from_spec(spec)
    b.set_state(spec.x0, spec.v0, 0)
    b.step(10)
    x, p, s = b.get_state()
    b.close()
    c = pimd.Context.from_spec(spec)
    c.set_state(x, p / spec.mass[None, :, None], s)
    c.step(10)
    xc, pc, sc = c.get_state()
    c.close()
    assert sc == sa == 20
    assert rel_err(xc, xa) <= TOL and rel_err(pc, pa) <= 1e-11


@pytest.mark.parametrize("integrator", [0, 1])
def test_noise_counter_across_the_32_bit_step_boundary(integrator):
    """The noise counter holds the step in two 32-bit words (OBABO's second O
    in the top bit of the upper one): a run from step 2^32 - 3 across 2^32,
    BAOAB and OBABO, matches the oracle started at the same step."""
    pimd = _pimd()
    spec = inputs.lj_liquid(n_atoms=108, n_beads=8, seed=9)
    spec.integrator = integrator
    s0 = 2**32 - 3
    _say("case %s integrator=%d from step %d" % (spec.name, integrator, s0))
    ctx = pimd.Context.from_spec(spec)
    ctx.set_state(spec.x0, spec.v0, s0)
    ctx.step(6)
    est = ctx.estimators()
    gx, gp, gs = ctx.get_state()
    ctx.close()
    st = oracle.State.from_spec(spec, step=s0)
    st.step(6)
    assert gs == s0 + 6
    check_states((gx, gp, gs, est), (st.x, st.p, int(st.step_count[0]), st.estimators(), st.sys))


# ------------------------------------------------------------ errors
def test_error_paths():
    pimd = _pimd()
    spec = inputs.harmonic_tiny(n_atoms=8, n_beads=4)
    ctx = pimd.Context.from_spec(spec)
    with pytest.raises(pimd.PimdError) as ei:
        ctx.step(1)
    assert ei.value.code == -4
    bad = spec.x0.copy()
    bad[0, 0, 0] = np.nan
    with pytest.raises(pimd.PimdError) as ei:
        ctx.set_state(bad, spec.v0)
    assert ei.value.code == -1
    with pytest.raises(pimd.PimdError) as ei:
        ctx.set_state(spec.x0, spec.v0, 2**63)
    assert ei.value.code == -1
    ctx.set_state(spec.x0, spec.v0, 2**63 - 1)
    ctx.set_state(spec.x0, spec.v0)
    with pytest.raises(pimd.PimdError):
        ctx.step(-1)
    ctx.close()
    # a huge time step drives the harmonic trap unstable -> non-finite flag
    s2 = inputs.harmonic_tiny(n_atoms=8, n_beads=4)
    s2.dt = 50.0
    s2.ensemble = inputs.NVE
    ctx = pimd.Context.from_spec(s2)
    ctx.set_state(s2.x0, s2.v0)
    ctx.step(400)
    with pytest.raises(pimd.PimdError) as ei:
        ctx.estimators()
    assert ei.value.code == -5
    ctx.close()
