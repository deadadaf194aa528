"""Serving: jobs that arrive while others run are admitted as slots free up,
share every tick with the running jobs, and each result equals the same job
run alone (bitwise: a system's arithmetic does not depend on its batch)."""
import numpy as np
import pytest

from paper_2602_13553_amd import inputs

pytestmark = pytest.mark.gpu


def small_trace():
    tr = inputs.serving_trace(n_jobs=10, rate=200.0, seed=11, n_range=(64, 400),
                              beads=(4, 8, 16, 32), steps_range=(5, 60))
    return tr


def test_served_results_equal_solo_runs():
    from paper_2602_13553_amd import serve
    tr = small_trace()
    rep = serve.serve(tr, max_active=3, tick=8, keep_states=True, realtime=False)
    assert len(rep.results) == len(tr)
    assert rep.max_active == 3           # jobs overlapped on the device
    seq = serve.serve_sequential(tr, keep_states=True, realtime=False)
    by_id = {r.job_id: r for r in seq.results}
    for r in rep.results:
        job = tr[r.job_id]
        s = by_id[r.job_id]
        print("job", r.job_id, job.kind, job.n_atoms, job.n_beads, job.nsteps, flush=True)
        assert r.step == s.step == job.nsteps
        assert np.array_equal(r.x, s.x) and np.array_equal(r.p, s.p), r.job_id
    # (replayed without waiting for arrival times, so latencies are not meaningful here)
    assert rep.summary()["jobs"] == len(tr)
