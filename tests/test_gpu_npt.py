"""GPU parity of the BZP barostat (NPT, NPH) against the oracle's NpT step:
positions, momenta, box, barostat velocity, the estimators and the enthalpy,
on identical seeded inputs and noise streams, through the C ABI."""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2602_13553_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_err(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _barostat(spec, ensemble, p_ext, tau_p, integrator=1):
    spec.ensemble, spec.integrator, spec.p_ext, spec.tau_p = ensemble, integrator, p_ext, tau_p
    return spec


def run_both(spec, chunks):
    from paper_2602_13553_amd import pimd
    n = sum(chunks)
    _say("case %s ensemble=%d N=%d P=%d steps=%d" % (spec.name, spec.ensemble, spec.n_atoms,
                                                      spec.n_beads, n))
    ctx = pimd.Context.from_spec(spec)
    ctx.set_state(spec.x0, spec.v0, 0)
    for c in chunks:
        ctx.step(c)
    est = ctx.estimators()
    gx, gp, gs = ctx.get_state()
    box, vw = ctx.barostat()
    ctx.close()
    st = oracle.State.from_spec(spec)
    st.step(n)
    return (gx, gp, gs, est, box, vw), st


def check(g, st, tol=TOL, est_tol=1e-10):
    gx, gp, gs, gest, gbox, gvw = g
    an = bool(st.sys.aniso)
    oest = st.estimators()
    ob = st.baro_energies()
    assert gs == int(st.step_count[0])
    ex, ep = rel_err(gx, st.x), rel_err(gp, st.p)
    W = oracle.lib().orc_baro_mass(oracle.C.byref(st.sys.cstruct()))
    vscale = math.sqrt(st.sys.n_beads * st.sys.kB * st.sys.temp / W)
    ovw = np.array(list(st.baro.vwa) if an else [st.baro.vw])
    gv = np.atleast_1d(np.asarray(gvw, dtype=np.float64))
    _say("  x rel %.3e  p rel %.3e  box %s / %s  vw %s / %s" %
         (ex, ep, np.array(gbox), np.array(st.box), gv, ovw))
    assert ex <= tol and ep <= tol, (ex, ep)
    for d in range(3):
        assert abs(gbox[d] / st.box[d] - 1) <= tol
    if not an:
        assert gbox[0] == gbox[1] == gbox[2]
    assert gv.shape == ovw.shape
    assert np.abs(gv - ovw).max() <= est_tol * max(np.abs(ovw).max(), vscale)
    scale = max(abs(oest["ekin"]), abs(oest["espring"]), abs(oest["epot"]))
    for name in ("ekin", "espring", "epot", "etot", "kprim", "kcv"):
        assert abs(gest[name] - oest[name]) <= est_tol * scale, (name, gest[name], oest[name])
    for name in ("pcv", "ppr", "pmd"):
        # the terms of each pressure are of the order of the energies over 3V
        assert abs(gest[name] - oest[name]) <= est_tol * 10 * scale / ob["volume"], name
    assert abs(gest["volume"] - ob["volume"]) <= tol * ob["volume"]
    hscale = scale + abs(ob["uw"]) + abs(ob["jw"]) + abs(ob["kw"])
    assert abs(gest["enthalpy"] - ob["enthalpy"]) <= est_tol * hscale
    if an:
        assert np.abs(np.array(gest["vwa"]) - ovw).max() <= est_tol * max(np.abs(ovw).max(), vscale)
        assert abs(gest["vw"] - ovw.mean()) <= est_tol * max(np.abs(ovw).max(), vscale)
    else:
        assert abs(gest["vw"] - st.baro.vw) <= est_tol * max(abs(st.baro.vw), vscale)
        assert gest["vwa"] == (0.0, 0.0, 0.0)


@pytest.mark.parametrize("ensemble", [2, 3])
def test_barostat_lj_matches_oracle(ensemble):
    spec = _barostat(inputs.lj_liquid(n_atoms=256, n_beads=8, seed=41), ensemble, 2.0, 0.2)
    g, st = run_both(spec, [1, 6, 3])
    check(g, st)


@pytest.mark.parametrize("ensemble", [2, 3])
def test_barostat_baoab_matches_oracle(ensemble):
    """The BAOAB splitting: A(dt/2), O(dt) on the beads and on v_W, A(dt/2)
    with the new v_W."""
    spec = _barostat(inputs.lj_liquid(n_atoms=256, n_beads=8, seed=50), ensemble, 2.0, 0.2,
                     integrator=0)
    g, st = run_both(spec, [1, 6, 3])
    check(g, st)
    spec = _barostat(inputs.water(n_atoms=384, n_beads=8, seed=51), ensemble, 0.5, 200.0,
                     integrator=0)
    g, st = run_both(spec, [4, 6])
    check(g, st)


@pytest.mark.parametrize("N,P", [(97, 3), (130, 6), (64, 1)])
def test_barostat_ragged_and_odd(N, P):
    """Bead counts that do not divide the block (ragged last tiles), and
    P = 1 (the classical NpT of the centroids alone)."""
    spec = _barostat(inputs.lj_liquid(n_atoms=N, n_beads=P, seed=48 + P), 2, 1.0, 0.3)
    g, st = run_both(spec, [3, 7])
    check(g, st)


@pytest.mark.parametrize("case", ["p8_high_pressure", "paper_example"])
def test_barostat_water_matches_oracle(case):
    """Water-shaped N = 384: at P = 8 under 0.5 kcal/mol/A^3 (about 3.5e4 bar,
    near the start's P_CV) with tau_p = 200 fs; and in the shape of the
    paper's NpT example: 128 molecules, P = 32, 300 K, 1 bar, dt 0.5 fs,
    PILE-L tau 100 fs, tau_p 500 fs."""
    if case == "p8_high_pressure":
        spec = _barostat(inputs.water(n_atoms=384, n_beads=8, seed=42), 2, 0.5, 200.0)
    else:
        spec = _barostat(inputs.water(n_atoms=384, n_beads=32, seed=46, dt=0.5, tau=100.0), 2,
                         1.0 / 69476.95, 500.0)
    g, st = run_both(spec, [2, 8])
    check(g, st)


def test_barostat_long_run_with_rebuilds():
    """200 steps under a fast barostat: the box shrinks by ~9% and the lists
    are rebuilt on the way; every bead pair inside rc must still be found
    (the oracle sums all pairs)."""
    spec = _barostat(inputs.lj_liquid(n_atoms=256, n_beads=4, seed=43), 2, 1.0, 0.1)
    g, st = run_both(spec, [64, 64, 72])
    _say("  rebuilds %d" % g[3]["n_rebuilds"])
    assert g[3]["n_rebuilds"] >= 2
    assert st.box[0] < 0.95 * spec.box[0]
    check(g, st, tol=1e-9, est_tol=1e-8)


def test_barostat_cell_lists_match_oracle():
    """A box of at least three centroid cells per dim (N = 2916): the lists
    are rebuilt from cells binned in the moving box, and each pair inside rc
    must still be found (the oracle sums all pairs)."""
    from paper_2602_13553_amd import pimd
    spec = _barostat(inputs.lj_liquid(n_atoms=2916, n_beads=4, seed=49), 2, 1.0, 0.1)
    ctx = pimd.Context.from_spec(spec)
    assert ctx.launch_info()["cells"] > 0
    ctx.close()
    g, st = run_both(spec, [16, 24])
    _say("  rebuilds %d" % g[3]["n_rebuilds"])
    assert g[3]["n_rebuilds"] >= 2
    check(g, st, tol=1e-10, est_tol=1e-9)


def test_barostat_running_sums_and_get_barostat_errors():
    from paper_2602_13553_amd import pimd
    spec = _barostat(inputs.lj_liquid(n_atoms=108, n_beads=4, seed=44), 2, 1.0, 0.3)
    ctx = pimd.Context.from_spec(spec)
    ctx.set_state(spec.x0, spec.v0, 0)
    ctx.step(5)
    e = ctx.estimators()
    ctx.close()
    st = oracle.State.from_spec(spec)
    acc = []
    for _ in range(5):
        st.step(1)
        acc.append(st.estimators()["etot"])
    assert e["count"] == 5
    assert abs(e["sum"]["etot"] - sum(acc)) <= 1e-10 * max(abs(a) for a in acc) * 5
    nvt = pimd.Context.from_spec(inputs.lj_liquid(n_atoms=108, n_beads=4, seed=44))
    nvt.set_state(spec.x0, spec.v0, 0)
    with pytest.raises(pimd.PimdError):
        nvt.barostat()
    nvt.close()


def test_barostat_checkpoint_restart():
    """20 steps in one go equal 10 steps, a checkpoint (state, box, v_W) and
    10 more steps in a new context."""
    from paper_2602_13553_amd import pimd
    spec = _barostat(inputs.lj_liquid(n_atoms=256, n_beads=8, seed=45), 2, 1.0, 0.2)
    a = pimd.Context.from_spec(spec)
    a.set_state(spec.x0, spec.v0, 0)
    a.step(20)
    xa, pa, sa = a.get_state()
    boxa, vwa = a.barostat()
    a.close()
    b = pimd.Context.from_spec(spec)
    b.set_state(spec.x0, spec.v0, 0)
    b.step(10)
    x, p, s = b.get_state()
    box, vw = b.barostat()
    b.close()
    c = pimd.Context.from_spec(spec)
    c.set_barostat(box, vw)
    c.set_state(x, p / spec.mass[None, :, None], s)
    c.step(10)
    xc, pc, sc = c.get_state()
    boxc, vwc = c.barostat()
    with pytest.raises(pimd.PimdError):
        c.set_barostat((1.0, 2.0, 1.0), 0.0)
    c.close()
    _say("  restart x rel %.3e p rel %.3e box %.3e vw %.3e" % (
        rel_err(xc, xa), rel_err(pc, pa), abs(boxc[0] / boxa[0] - 1), abs(vwc - vwa)))
    assert sc == sa == 20
    assert rel_err(xc, xa) <= TOL and rel_err(pc, pa) <= 1e-11
    assert abs(boxc[0] / boxa[0] - 1) <= TOL
    assert abs(vwc - vwa) <= 1e-10 * max(abs(vwa), 1e-3)


def test_barostat_full_size_nph_conserves_the_enthalpy():
    """The LJ liquid at full size (N = 4000, P = 32), where the oracle cannot
    follow: in NpH the enthalpy H + K_W + U_W + J_W is a constant of the
    motion, so its spread must fall about fourfold when dt halves (measured:
    3.0 from dt = 0.002 to 0.001, 4.0 from 0.001 to 0.0005, over one time
    unit), and stay within a few times the NVE energy's spread at the same
    dt (measured: 3.0 times), while the volume moves by ~40%.  rc = 3 keeps
    the force's jump at the cutoff small."""
    from paper_2602_13553_amd import pimd

    def run(dt, ensemble, t_total=1.0):
        spec = inputs.lj_liquid(seed=47)
        spec.lj_rc, spec.dt = 3.0, dt
        if ensemble == 3:
            spec = _barostat(spec, 3, 1.0, 0.5)
        else:
            spec.ensemble, spec.integrator = 1, 1
        ctx = pimd.Context.from_spec(spec)
        ctx.set_state(spec.x0, spec.v0, 0)
        h, v = [], []
        n = int(round(t_total / dt))
        for _ in range(n // 20):
            ctx.step(20)
            e = ctx.estimators()
            h.append(e["enthalpy"] if ensemble == 3 else e["etot"])
            v.append(e["volume"])
        ctx.close()
        return np.ptp(h), (max(v) / min(v) if ensemble == 3 else 1.0)

    h1, vr = run(0.001, 3)
    h2, _ = run(0.0005, 3)
    e2, _ = run(0.0005, 1)
    _say("  enthalpy spread dt=0.001: %.4e  dt=0.0005: %.4e  NVE: %.4e  V ratio %.3f" %
         (h1, h2, e2, vr))
    assert vr > 1.2
    assert 3.0 < h1 / h2 < 5.0
    assert h2 < 5.0 * e2


# ------------------------------------------- anisotropic barostat (App. E)

def _stretch(spec, f):
    """The same lattice in a rectangular box: coordinates and box lengths
    scaled by f per dimension."""
    spec.x0 = np.ascontiguousarray(spec.x0 * np.asarray(f)[None, None, :])
    spec.box = tuple(b * s for b, s in zip(spec.box, f))
    return spec


def _aniso(spec, ensemble, p_ext, tau_p, integrator=1):
    spec = _barostat(spec, ensemble, p_ext, tau_p, integrator)
    spec.baro_aniso = 1
    return spec


@pytest.mark.parametrize("ensemble", [2, 3])
@pytest.mark.parametrize("integrator", [0, 1])
def test_aniso_barostat_lj_matches_oracle(ensemble, integrator):
    """One v_W per dimension in a rectangular box (the stress differs per
    dimension, so the three lengths part): positions, momenta, the three
    lengths and velocities, the estimators and the enthalpy."""
    spec = _stretch(inputs.lj_liquid(n_atoms=256, n_beads=8, seed=60 + integrator), (1.0, 0.92, 1.12))
    spec = _aniso(spec, ensemble, 2.0, 0.2, integrator)
    g, st = run_both(spec, [1, 6, 3])
    check(g, st)
    assert len(set(g[4])) == 3


def test_aniso_barostat_water_matches_oracle():
    """Water-shaped N = 384, P = 8, BAOAB: the bonds' share of each
    dimension's virial (an O atom's lanes also write its H atoms' forces)."""
    spec = _aniso(inputs.water(n_atoms=384, n_beads=8, seed=62), 2, 0.5, 200.0, integrator=0)
    g, st = run_both(spec, [4, 6])
    check(g, st)


@pytest.mark.parametrize("N,P", [(97, 3), (64, 1)])
def test_aniso_barostat_ragged_and_odd(N, P):
    spec = _stretch(inputs.lj_liquid(n_atoms=N, n_beads=P, seed=63 + P), (1.1, 1.0, 0.95))
    spec = _aniso(spec, 2, 1.0, 0.3)
    g, st = run_both(spec, [3, 7])
    check(g, st)


def test_aniso_barostat_cell_lists_and_rebuilds():
    """N = 2916 in a rectangular box under a fast barostat: cells binned in a
    box whose three lengths scale apart, rebuilds against the smallest
    scaling; every pair inside rc must still be found (the oracle sums all
    pairs)."""
    from paper_2602_13553_amd import pimd
    spec = _stretch(inputs.lj_liquid(n_atoms=2916, n_beads=4, seed=64), (1.0, 1.08, 0.94))
    spec = _aniso(spec, 2, 1.0, 0.1)
    ctx = pimd.Context.from_spec(spec)
    assert ctx.launch_info()["cells"] > 0
    ctx.close()
    g, st = run_both(spec, [16, 24])
    _say("  rebuilds %d" % g[3]["n_rebuilds"])
    assert g[3]["n_rebuilds"] >= 2
    check(g, st, tol=1e-10, est_tol=1e-9)


def test_aniso_barostat_checkpoint_restart():
    """20 steps in one go equal 10 steps, a checkpoint (state, three lengths,
    three v_Wa) and 10 more in a new context; the anisotropic barostat takes
    any box of positive lengths and exactly three velocities."""
    from paper_2602_13553_amd import pimd
    spec = _stretch(inputs.lj_liquid(n_atoms=256, n_beads=8, seed=65), (1.0, 1.0, 1.1))
    spec = _aniso(spec, 2, 1.0, 0.2, integrator=0)
    a = pimd.Context.from_spec(spec)
    a.set_state(spec.x0, spec.v0, 0)
    a.step(20)
    xa, pa, sa = a.get_state()
    boxa, vwa = a.barostat()
    a.close()
    b = pimd.Context.from_spec(spec)
    b.set_state(spec.x0, spec.v0, 0)
    b.step(10)
    x, p, s = b.get_state()
    box, vw = b.barostat()
    b.close()
    assert isinstance(vw, tuple) and len(vw) == 3
    c = pimd.Context.from_spec(spec)
    with pytest.raises(ValueError):
        c.set_barostat(box, 0.0)
    with pytest.raises(pimd.PimdError):
        c.set_barostat(box, (0.0, float("nan"), 0.0))
    with pytest.raises(pimd.PimdError):
        c.set_barostat((box[0], -1.0, box[2]), vw)
    c.set_barostat(box, vw)
    c.set_state(x, p / spec.mass[None, :, None], s)
    c.step(10)
    xc, pc, sc = c.get_state()
    boxc, vwc = c.barostat()
    c.close()
    _say("  restart x rel %.3e p rel %.3e box %s / %s" % (rel_err(xc, xa), rel_err(pc, pa), boxc, boxa))
    assert sc == sa == 20
    assert rel_err(xc, xa) <= TOL and rel_err(pc, pa) <= 1e-11
    for d in range(3):
        assert abs(boxc[d] / boxa[d] - 1) <= TOL
        assert abs(vwc[d] - vwa[d]) <= 1e-10 * max(abs(vwa[d]), 1e-3)
