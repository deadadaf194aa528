"""Continuous-batching server for PIMD jobs on one GPU.

Jobs (a system, its initial state and a number of steps) arrive over time.
A job is admitted as soon as a slot and device memory (by
``pimd_workspace_bytes``) are free; every admitted job then advances inside
one shared ``pimd_batch`` whose step is a fixed handful of launches for all
jobs together.  Each job carries its own step budget on the device, so jobs of
different lengths share every tick and simply stop when their budget is spent.
Finished jobs are read back and retired at tick boundaries, which frees their
slot and memory for waiting jobs.

``serve(trace)`` replays a timed trace (``inputs.serving_trace``) in real time
and reports time-to-result percentiles and aggregate bead*atom*steps/s.
``serve_sequential(trace)`` is the one-job-at-a-time reference: the same jobs,
each run alone with ``pimd_step`` in arrival order.
"""
from __future__ import annotations

import collections
import ctypes as C
import queue
import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import pimd


@dataclass
class JobResult:
    job_id: int
    arrival: float
    admitted: float
    finished: float
    bead_atom_steps: int
    x: np.ndarray | None = None
    p: np.ndarray | None = None
    step: int = 0

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclass
class ServeReport:
    results: list = field(default_factory=list)
    wall: float = 0.0
    ticks: int = 0
    max_active: int = 0

    def summary(self) -> dict:
        lat = np.array([r.latency for r in self.results]) if self.results else np.zeros(1)
        work = sum(r.bead_atom_steps for r in self.results)
        return {"jobs": len(self.results), "p50_s": float(np.percentile(lat, 50)),
                "p99_s": float(np.percentile(lat, 99)), "mean_s": float(lat.mean()),
                "bead_atom_steps_per_s": work / self.wall if self.wall > 0 else 0.0,
                "wall_s": self.wall, "ticks": self.ticks, "max_active": self.max_active}


class _Prefetch:
    """Builds job specs (host-side initial states) ahead of their arrival."""

    def __init__(self, jobs, depth: int = 24):
        self._q = queue.Queue(maxsize=depth)
        self._t = threading.Thread(target=self._run, args=(list(jobs),), daemon=True)
        self._t.start()

    def _run(self, jobs):
        for j in jobs:
            self._q.put((j, j.spec()))
        self._q.put(None)

    def get(self):
        return self._q.get()


def workspace_bytes(spec) -> int:
    lib = pimd.load()
    p = pimd.params_from_spec(spec)
    keep = []
    topo = pimd._topology(spec.lj_active, spec.bonds, keep)
    mass = np.ascontiguousarray(spec.mass, dtype=np.float64)
    n = C.c_size_t()
    rc = lib.pimd_workspace_bytes(C.byref(p), pimd._dp(mass),
                                  C.byref(topo) if topo is not None else None, C.byref(n))
    if rc != 0:
        raise pimd.PimdError(rc, lib.pimd_last_error(None).decode())
    return int(n.value)


def serve(trace, hbm_budget: float = 200e9, max_active: int = 64, tick: int = 32,
          keep_states: bool = False, realtime: bool = True,
          max_active_bead_atoms: float = 2e6, progress=None) -> ServeReport:
    """Replay ``trace`` (jobs with arrival times in seconds) through one batch.

    Admission is first-come first-served under three limits: the slot count,
    the HBM budget (``pimd_workspace_bytes`` of the running jobs) and the
    bead*atoms stepped together.  The last one stops admitting once the GPU
    is saturated: beyond it, another job only slows every running job down
    (shared throughput) instead of raising the aggregate rate, so waiting
    jobs start later but every job finishes sooner.  A job is always admitted
    when nothing runs.  progress: called with the number of finished jobs
    each time a tick finishes some."""
    batch = pimd.Batch()
    pre = _Prefetch(sorted(trace, key=lambda j: j.arrival))
    report = ServeReport()
    waiting = collections.deque()          # (job, spec) arrived, not admitted
    upcoming = None                        # next (job, spec) from the prefetcher
    exhausted = False
    running = {}                           # sid -> (job, bytes, admitted time)
    left = {}                              # sid -> steps still in its budget
    used = 0.0
    active_ba = 0
    t0 = time.perf_counter()

    def now():
        return time.perf_counter() - t0

    while True:
        # arrivals up to now (or all of them when not replaying in real time)
        while not exhausted:
            if upcoming is None:
                item = pre.get()
                if item is None:
                    exhausted = True
                    break
                upcoming = item
            if realtime and upcoming[0].arrival > now():
                break
            waiting.append(upcoming)
            upcoming = None
        # admission: FIFO, while a slot and the memory budget allow
        while waiting and len(running) < max_active:
            job, spec = waiting[0]
            nbytes = workspace_bytes(spec)
            ba = job.n_atoms * job.n_beads
            if running and (used + nbytes > hbm_budget or active_ba + ba > max_active_bead_atoms):
                break
            waiting.popleft()
            sid = batch.add(spec)
            batch.set_state(sid, spec.x0, spec.v0, 0)
            batch.set_budget(sid, job.nsteps)
            running[sid] = (job, nbytes, now())
            left[sid] = job.nsteps
            used += nbytes
            active_ba += ba
        report.max_active = max(report.max_active, len(running))
        if not running:
            if exhausted and not waiting:
                break
            if upcoming is not None and realtime:
                time.sleep(max(0.0, min(0.01, upcoming[0].arrival - now())))
            continue
        # one tick for every running job.  A tick takes min(tick, budget left)
        # steps of each job, so the host knows which jobs it finishes without
        # reading the device; the tick is waited for (once) only when it
        # finishes one, and each finished job's step count is checked then.
        batch.step(tick)
        report.ticks += 1
        done = []
        for sid in running:
            left[sid] -= tick
            if left[sid] <= 0:
                done.append(sid)
        if not done:
            continue
        for sid in done:
            e = batch.estimators(sid)
            assert e["step"] == running[sid][0].nsteps, (e["step"], running[sid][0].nsteps)
        t_done = now()
        for sid in done:
            left.pop(sid)
            job, nbytes, adm = running.pop(sid)
            r = JobResult(job.job_id, job.arrival, adm, t_done,
                          job.n_atoms * job.n_beads * job.nsteps)
            if keep_states:
                r.x, r.p, r.step = batch.get_state(sid)
            batch.remove(sid)
            used -= nbytes
            active_ba -= job.n_atoms * job.n_beads
            report.results.append(r)
        if progress is not None:
            progress(len(report.results))
    report.wall = now()
    batch.close()
    return report


def serve_sequential(trace, keep_states: bool = False, realtime: bool = True,
                     progress=None) -> ServeReport:
    """One job at a time, in arrival order, each with its own context;
    progress: called with the number of finished jobs after each."""
    report = ServeReport()
    pre = _Prefetch(sorted(trace, key=lambda j: j.arrival))
    t0 = time.perf_counter()
    while True:
        item = pre.get()
        if item is None:
            break
        job, spec = item
        if realtime:
            wait = job.arrival - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
        adm = time.perf_counter() - t0
        ctx = pimd.Context.from_spec(spec, use_torch_workspace=False)
        ctx.set_state(spec.x0, spec.v0, 0)
        ctx.step(job.nsteps)
        e = ctx.estimators()
        r = JobResult(job.job_id, job.arrival, adm, time.perf_counter() - t0,
                      job.n_atoms * job.n_beads * job.nsteps)
        if keep_states:
            r.x, r.p, r.step = ctx.get_state()
        assert e["step"] == job.nsteps
        ctx.close()
        report.results.append(r)
        if progress is not None:
            progress(len(report.results))
    report.wall = time.perf_counter() - t0
    report.max_active = 1
    return report
