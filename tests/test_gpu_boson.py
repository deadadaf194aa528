"""GPU parity of the bosonic exchange springs (pimd_boson_spring, through the
C ABI) against the oracle's recursion (in extended precision): V_B, the
primitive estimator's weighted ring energy EV_B, the forces and the link
probabilities, element by element.

Bar: 1e-12, relative for V_B and EV_B, relative to the largest force for the
forces, absolute for the probabilities.  The kernels run the recursion over
the links alone (the inner-ring energies enter every term equally and are
added at the end) with double-double chain sums and V', so the exponent of
every ring weight carries the rounding of its own size, independent of
V_B's."""
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

BAR = 1e-12


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _cloud(N, P, seed, spread=1.2, box=None):
    rng = np.random.default_rng(seed)
    if box is None:
        return rng.normal(0, 0.4, (P, N, 3)) + rng.normal(0, spread, (1, N, 3))
    # unwrapped rings around centers spread over the box
    return rng.normal(0, 0.4, (P, N, 3)) + rng.uniform(0, 1, (1, N, 3)) * np.asarray(box)


def _compare(x, k, b, box=None):
    from paper_2602_13553_amd import pimd
    v, ev, f, prob = pimd.boson_spring(x, k, b, box=box)
    f, prob = f.cpu().numpy(), prob.cpu().numpy()
    vo, fo, po, evo = oracle.boson_spring(x, k, b, with_ev=True, box=box)
    ef = np.abs(f - fo).max() / max(np.abs(fo).max(), 1e-300)
    ep = np.abs(prob - po).max()
    _say("  V %.15e / %.15e  EV %.15e / %.15e  f rel %.3e  prob %.3e"
         % (v, vo, ev, evo, ef, ep))
    assert abs(v - vo) <= BAR * max(1.0, abs(vo)), (v, vo)
    assert abs(ev - evo) <= BAR * max(1.0, abs(evo)), (ev, evo)
    assert ef <= BAR, ef
    assert ep <= BAR, ep


@pytest.mark.parametrize("N,P", [(1, 4), (2, 1), (3, 8), (17, 32), (64, 16), (300, 4),
                                 (512, 2), (700, 3), (1024, 2)])
def test_boson_spring_matches_oracle(N, P):
    """Particles spread over a few thermal lengths, so that exchange matters;
    N up to the library's limit, with ragged thread counts in every stage."""
    x = _cloud(N, P, N * 131 + P)
    _say("case boson N=%d P=%d" % (N, P))
    _compare(x, 1.1, 0.9)


@pytest.mark.parametrize("N,P,L", [(5, 4, 2.0), (64, 8, 4.0), (400, 2, 8.0)])
def test_boson_spring_periodic_matches_oracle(N, P, L):
    """Links under the minimum image in a periodic box small enough that
    many of them cross a face."""
    box = [L, L * 1.1, L * 0.9]
    x = _cloud(N, P, 7 * N + P, box=box)
    _say("case boson periodic N=%d P=%d L=%g" % (N, P, L))
    _compare(x, 1.1, 0.9, box=box)


def test_boson_spring_stiff_springs():
    """Stiff springs and a large beta_n: the ring weights span many orders
    of magnitude (V_B ~ 1e4), where differences of plain prefix sums would
    lose the 1e-12 bar."""
    x = _cloud(256, 4, 3, spread=3.0)
    _say("case boson stiff N=256 P=4")
    _compare(x, 20.0, 2.0)


def test_boson_spring_errors():
    from paper_2602_13553_amd import pimd
    with pytest.raises(pimd.PimdError) as ei:
        pimd.boson_spring(np.zeros((2, 1025, 3)), 1.0, 1.0)
    assert ei.value.code == pimd.PIMD_ERR_UNSUPPORTED
    with pytest.raises(pimd.PimdError) as ei:
        pimd.boson_spring(np.zeros((2, 3, 3)), 1.0, 0.0)
    assert ei.value.code == pimd.PIMD_ERR_ARG
    with pytest.raises(pimd.PimdError):
        pimd.boson_spring(np.zeros((2, 3, 3)), 1.0, 1.0, box=[1.0, -1.0, 1.0])
