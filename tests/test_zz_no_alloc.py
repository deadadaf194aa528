"""The allocation-free bosonic exchange entry point (pimd_boson_spring_noalloc,
through the C ABI) against pimd_boson_spring on the same inputs: two calls
in a row on the library's static scratch, the second with a smaller input, so
that the second call runs over what the first left in the scratch."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _cloud(N, P, seed, box=None):
    rng = np.random.default_rng(seed)
    if box is None:
        return rng.normal(0, 0.4, (P, N, 3)) + rng.normal(0, 1.2, (1, N, 3))
    return rng.normal(0, 0.4, (P, N, 3)) + rng.uniform(0, 1, (1, N, 3)) * np.asarray(box)


def _check(a, b):
    """noalloc result a against the allocating entry point's b: the same
    kernels on the same inputs, so equal to the parity bar (1e-12) and in
    practice bit for bit."""
    va, eva, fa, pa = a
    vb, evb, fb, pb = b
    fa, fb, pa, pb = fa.cpu().numpy(), fb.cpu().numpy(), pa.cpu().numpy(), pb.cpu().numpy()
    _say("  V %.17g / %.17g  EV %.17g / %.17g  max|df| %.3e  max|dprob| %.3e"
         % (va, vb, eva, evb, np.abs(fa - fb).max(), np.abs(pa - pb).max()))
    assert abs(va - vb) <= 1e-12 * max(1.0, abs(vb))
    assert abs(eva - evb) <= 1e-12 * max(1.0, abs(evb))
    assert np.abs(fa - fb).max() <= 1e-12 * max(np.abs(fb).max(), 1e-300)
    assert np.abs(pa - pb).max() <= 1e-12


def test_noalloc_matches_allocating_entry_point_twice():
    from paper_2602_13553_amd import pimd
    import torch
    cases = [(512, 8, None, 1), (100, 3, [3.0, 3.3, 2.7], 2)]
    for N, P, box, seed in cases:
        _say("case noalloc N=%d P=%d box=%s" % (N, P, box))
        x = torch.tensor(_cloud(N, P, seed, box), dtype=torch.float64, device="cuda")
        a = pimd.boson_spring(x, 1.1, 0.9, box=box, noalloc=True)
        b = pimd.boson_spring(x, 1.1, 0.9, box=box)
        _check(a, b)


def test_noalloc_limit():
    from paper_2602_13553_amd import pimd
    with pytest.raises(pimd.PimdError) as ei:
        pimd.boson_spring(np.zeros((2, 513, 3)), 1.0, 1.0, noalloc=True)
    assert ei.value.code == pimd.PIMD_ERR_UNSUPPORTED
