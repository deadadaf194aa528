"""GPU parity of the bosonic exchange spring kernel (pimd_boson_spring, through
the C ABI) against the oracle's recursion: V_B, the forces and the link
probabilities, element by element.

Bar: V_B to 1e-12 relative.  The kernel forms each ring energy as a
difference of prefix sums, whose rounding is about eps * V_B in absolute
terms, against the oracle's direct sums; every ring's weight
exp(-beta_n (E + V - V)) then carries a relative error of about
beta_n * eps * V_B.  The probabilities (absolute) and the forces (relative to
their largest) are held to max(1e-12, 20 beta_n eps V_B)."""
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("N,P", [(1, 4), (2, 1), (3, 8), (17, 32), (64, 16), (300, 4), (512, 2)])
def test_boson_spring_matches_oracle(N, P):
    from paper_2602_13553_amd import pimd
    rng = np.random.default_rng(N * 131 + P)
    # particles spread over a few thermal lengths, so that exchange matters
    x = rng.normal(0, 0.4, (P, N, 3)) + rng.normal(0, 1.2, (1, N, 3))
    k, b = 1.1, 0.9
    _say("case boson N=%d P=%d" % (N, P))
    v, f, prob = pimd.boson_spring(x, k, b)
    f, prob = f.cpu().numpy(), prob.cpu().numpy()
    vo, fo, po = oracle.boson_spring(x, k, b)
    ef = np.abs(f - fo).max() / max(np.abs(fo).max(), 1e-300)
    _say("  V %.15e / %.15e  f rel %.3e  prob %.3e" % (v, vo, ef, np.abs(prob - po).max()))
    bar = max(1e-12, 20 * b * np.finfo(float).eps * abs(vo))
    assert abs(v - vo) <= 1e-12 * max(1.0, abs(vo))
    assert ef <= bar, (ef, bar)
    assert np.abs(prob - po).max() <= bar, (np.abs(prob - po).max(), bar)


def test_boson_spring_errors():
    from paper_2602_13553_amd import pimd
    with pytest.raises(pimd.PimdError):
        pimd.boson_spring(np.zeros((2, 513, 3)), 1.0, 1.0)
    with pytest.raises(pimd.PimdError):
        pimd.boson_spring(np.zeros((2, 3, 3)), 1.0, 0.0)


@pytest.mark.parametrize("N,P,thermo", [(3, 8, True), (5, 4, False), (1, 1, True), (40, 16, True)])
def test_boson_step_matches_oracle(N, P, thermo):
    """The bosonic Cartesian step (pimd_boson_step) against the oracle's
    orc_boson_step: 20 steps of trapped bosons, positions and velocities
    element by element, V_B and the beads' trap energies."""
    from paper_2602_13553_amd import pimd
    rng = np.random.default_rng(7 * N + P)
    dt, tau, hbar, omega, seed = 0.005, 0.1, 0.5, 1.0, 11
    x = rng.normal(0, 0.8, (1, N, 3)) + rng.normal(0, 0.2, (P, N, 3))
    v = rng.normal(0, np.sqrt(P), (P, N, 3))
    _say("case boson step N=%d P=%d thermostat=%d" % (N, P, thermo))
    gx, gv, gf, gu, gvb = pimd.boson_step(x, v, 1.0, 1.0, 1.0, hbar, 1.0, dt, tau, omega, seed,
                                          thermo, 0, 20)
    gx, gv, gu = gx.cpu().numpy(), gv.cpu().numpy(), gu.cpu().numpy()
    s = oracle.System(n_atoms=N, n_beads=P, mass=np.ones(N), temp=1.0, hbar=hbar, dt=dt, tau=tau,
                      nve=not thermo, pot=oracle.POT_HARMONIC, omega=omega, seed=seed)
    st = oracle.BosonState(s, x, v)
    st.step(20)
    ex = np.abs(gx - st.x).max() / np.abs(st.x).max()
    ev = np.abs(gv - st.v).max() / np.abs(st.v).max()
    _say("  x rel %.3e  v rel %.3e  V_B %.12e / %.12e" % (ex, ev, gvb, st.vb[0]))
    assert ex <= 1e-12 and ev <= 1e-12
    assert abs(gvb - st.vb[0]) <= 1e-12 * max(1.0, abs(st.vb[0]))
    assert np.abs(gu.sum(axis=1) - st.U).max() <= 1e-12 * max(1.0, np.abs(st.U).max())
