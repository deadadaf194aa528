"""Throughput of the ring-polymer BAOAB + PILE-L step on one MI355X.

One step = the whole hot path over one batch of synthetic input: normal-mode
transforms, B/A/O/A/B, PILE-L noise, bead-batched forces, estimators.  The
headline workload is the water-shaped system (N=32766 atoms: O-H harmonic
bonds plus O-O LJ at 9 A, 1 g/cm^3, 300 K, P=64 beads, dt=0.25 fs, PILE-L
tau=100 fs), the shape of the paper's DP water runs.  Legs beside it: the
same system at P=32, the LJ quantum liquid (N=4000, P=32), the step pass on a
working set far beyond the 256 MB Infinity Cache (the water-shaped system
four times larger, N=131070, P=64), a plain-copy HBM probe, and the CPU
oracle on the host cores at one thread and at every core.

Prints ONE JSON line: bead*atom*steps/s over exactly --steps timed steps
(after --warmup untimed ones), the roofline of the dominant kernel from HIP
events on the library's stream, and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2602_13553_amd import inputs  # noqa: E402

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 vector (256 CU x 2.4 GHz x 128 flop/clk)
LJ_FLOPS_PER_PAIR = 23         # per ordered bead pair inside rc (full neighbor list)
FUSED_BYTES_PAIR = 120         # per bead*atom: read x, v~, f; write x, v~ (FP64 x 3 dims)
FUSED_BYTES_EXT = 96           # per bead*atom with in-kernel trap forces (no f array)


WORKLOADS = {
    "lj": ("LJ quantum liquid, N=4000, P=32, rho=0.8", inputs.lj_liquid,
           "synthetic (seeded FCC LJ liquid, Maxwell-Boltzmann bead velocities at P*T)"),
    "water32": ("water-shaped, N=32766, P=32", lambda: inputs.water(n_beads=32),
                "synthetic (seeded water-shaped O/H lattice, Maxwell-Boltzmann bead velocities at P*T)"),
    "water64": ("water-shaped, N=32766, P=64", lambda: inputs.water(n_beads=64),
                "synthetic (seeded water-shaped O/H lattice, Maxwell-Boltzmann bead velocities at P*T)"),
    "water64x4": ("water-shaped, N=131070, P=64 (the N=32766 system four times larger at the "
                  "same density)", lambda: inputs.water(n_atoms=131072, n_beads=64),
                  "synthetic (seeded water-shaped O/H lattice, Maxwell-Boltzmann bead velocities at P*T)"),
    "harmonic": ("harmonic oscillators, N=64, P=4", inputs.harmonic_tiny,
                 "synthetic (seeded Gaussian positions, Maxwell-Boltzmann bead velocities at P*T)"),
}


PROFILES = os.path.join(ROOT, "profiles")
# the kernel sources a profile's counters belong to (host-side code excluded)
KERNEL_SOURCES = ("pimd_device.h", "pimd_fused_mfma.hip", "pimd_internal.h", "pimd_kernels.hip",
                  "pimd_tuning.h")


# committed rocprofv3 summaries by (workload, kernel)
PROFILE_FILES = {
    ("lj", "k_pair"): "k_pair_lj_n4000_p32.txt",
    ("lj", "k_fused<false>"): "k_fused_lj_n4000_p32.txt",
    ("water64", "k_fused_mfma<64, false, false>"): "k_fused_mfma_water_n32766_p64.txt",
    ("water64", "k_pair"): "k_pair_water_n32766_p64.txt",
    ("water64x4", "k_fused_mfma<64, false, false>"): "k_fused_mfma_water_n131070_p64.txt",
    ("water64x4", "k_pair"): "k_fused_mfma_water_n131070_p64.txt",
}


def _counter_name(kname: str) -> str:
    """The kernel's name as rocprofv3 prints it."""
    return "void pimd::%s" % kname if "<" in kname else "pimd::%s(" % kname


def kernel_source_sha256() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2602_13553_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profiled_traffic(fname: str, kernel: str):
    """HBM bytes per launch of `kernel` from a committed rocprofv3 summary
    (FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by what the counter
    reads for a plain copy of known size), or None when there is none or the
    kernel sources have changed since the counters were taken."""
    try:
        with open(os.path.join(PROFILES, fname)) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return None
    for ln in lines:
        if ln.startswith("traffic " + kernel):
            kv = dict(t.split("=", 1) for t in ln.split() if "=" in t)
            if kv.get("source_sha256") != kernel_source_sha256():
                return None
            return int(kv["total_bytes"])
    return None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def pairs_inside_cutoff(x, box, rc, active=None):
    """Ordered bead pairs (i, j), i != j, of the same bead with |r_ij| < rc under
    the minimum image (scipy cKDTree with periodic box), summed over beads."""
    from scipy.spatial import cKDTree
    L = np.asarray(box)
    tot = 0
    for k in range(x.shape[0]):
        pts = x[k] if active is None else x[k][np.asarray(active).astype(bool)]
        tree = cKDTree(np.mod(pts, L), boxsize=L)
        tot += 2 * len(tree.query_pairs(rc, output_type="ndarray"))
    return tot


def sync(ctx):
    import torch
    torch.cuda.synchronize()
    return ctx.estimators()


def bench_boson():
    """The bosonic exchange springs (energy, estimator energy, forces, link
    probabilities) per call, on N particles of P beads spread over a few
    thermal lengths; each call allocates and frees its scratch and waits for
    its stream."""
    import torch
    from paper_2602_13553_amd import pimd
    out = {}
    for N, P in ((64, 32), (512, 8), (1024, 8)):
        rng = np.random.default_rng(N + P)
        x = torch.tensor(rng.normal(0, 0.4, (P, N, 3)) + rng.normal(0, 1.2, (1, N, 3)),
                         dtype=torch.float64, device="cuda")
        for _ in range(3):
            pimd.boson_spring(x, 1.1, 0.9)
        n = 50
        t0 = time.perf_counter()
        for _ in range(n):
            pimd.boson_spring(x, 1.1, 0.9)
        out["N%d_P%d_us_per_call" % (N, P)] = (time.perf_counter() - t0) / n * 1e6
    return out


def bench_bosons():
    """Bosonic contexts (the bosonic fix's Cartesian step with the exchange
    springs in every step): 1024 trapped bosons at P = 32, and an LJ liquid
    of 500 bosons at P = 32 (helium-like reduced units)."""
    out = {}
    for name, spec in (("trap_n1024_p32", inputs.trapped_bosons(n_atoms=1024, n_beads=32)),
                       ("lj_n500_p32", inputs.lj_bosons(n_atoms=500, n_beads=32))):
        ms, _, prof, _, _, _ = run_gpu(spec, 200, 20, 50)
        out[name] = {"workload": spec.name, "ms_per_step": ms,
                     "bead_atom_steps_per_s": spec.bead_atoms * 1e3 / ms,
                     "kernels_ms": {k: v[0] for k, v in kernel_avgs(prof).items()}}
    return out


def bench_npt(make):
    """The barostat's step (two passes with their finalizes, then the forces
    in the new box) on the LJ liquid, and on the shape of the paper's NpT
    example: 128 water molecules, P = 32, 300 K, dt 0.5 fs, PILE-L tau 0.1 ps,
    BZP tau_p 0.5 ps at 1 bar (water-shaped potential in place of its DP
    model)."""
    out = {}
    lj = make()
    lj.integrator, lj.ensemble, lj.p_ext, lj.tau_p = 1, inputs.NPT, 0.5, 0.5
    ms, _, prof, _, _, _ = run_gpu(lj, 500, 50, 100)
    out["lj"] = {"workload": "LJ quantum liquid, N=%d, P=%d, NpT (OBABO + BZP, p_ext=0.5, tau_p=0.5)"
                             % (lj.n_atoms, lj.n_beads),
                 "ms_per_step": ms, "bead_atom_steps_per_s": lj.bead_atoms * 1e3 / ms,
                 "kernels_ms": {k: v[0] for k, v in kernel_avgs(prof).items()}}
    w = inputs.water(n_atoms=384, n_beads=32, dt=0.5, tau=100.0)
    bar = 1.0 / 69476.95                   # kcal/mol/A^3
    w.integrator, w.ensemble, w.p_ext, w.tau_p = 1, inputs.NPT, bar, 500.0
    ms, _, prof, _, _, _ = run_gpu(w, 1000, 100, 100)
    out["water_128"] = {"workload": "128 water molecules (N=384), P=32, NpT at 300 K and 1 bar, "
                                    "dt 0.5 fs (the paper's NpT example's shape)",
                        "ms_per_step": ms, "ns_per_day": 0.5e-6 * 86400.0 * 1e3 / ms,
                        "kernels_ms": {k: v[0] for k, v in kernel_avgs(prof).items()}}
    return out


def run_gpu(spec, steps, warmup, profile_steps, flags=0):
    from paper_2602_13553_amd import pimd
    ctx = pimd.Context.from_spec(spec, flags=flags)
    ctx.set_state(spec.x0, spec.v0, 0)
    ctx.step(warmup)
    sync(ctx)
    t0 = time.perf_counter()
    ctx.step(steps)
    est = sync(ctx)
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / steps
    # profiled region: same workload, per-kernel HIP events on the library stream
    ctx.profile_begin()
    t2 = time.perf_counter()
    ctx.step(profile_steps)
    prof = ctx.profile_end()
    t3 = time.perf_counter()
    x, p, s = ctx.get_state()
    info = ctx.launch_info()
    ctx.close()
    return ms_step, est, prof, (t3 - t2) * 1e3 / profile_steps, x, info


def kernel_avgs(prof):
    return {k: (ms / n if n else 0.0, n) for k, (n, ms) in prof.items()}


def _omp_threads(n: int) -> None:
    """Thread count of the OpenMP runtime the oracle runs on (libgomp), for
    the parallel regions that follow."""
    import ctypes
    ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))


def host_cores() -> int:
    """Host threads this process may use: OMP_NUM_THREADS when set (the box's
    CPU share), else the CPU affinity mask."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    return len(os.sched_getaffinity(0))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_one(spec, threads: int, max_seconds: float, max_steps: int = 200):
    """The oracle as it stands, at `threads` OpenMP threads, on a bounded
    sample of the workload: steps from its initial state (the forces of the
    initial state, computed when the state is set up, are outside the
    timing) until max_seconds, at least one."""
    import oracle
    _omp_threads(threads)
    st = oracle.State.from_spec(spec)
    n, t = 0, 0.0
    while n < max_steps:
        t0 = time.perf_counter()
        st.step(1)
        t += time.perf_counter() - t0
        n += 1
        if t * (n + 1) / n > max_seconds:
            break
    return {"value": spec.bead_atoms * n / t, "unit": "bead*atom*steps/s", "cores": threads,
            "kind": "oracle",
            "sample": "%d step(s) of %s from its initial state, %.1f s" % (n, spec.name, t)}


def cpu_baseline(spec, legs):
    """The oracle on the host cores: the headline workload at every core and
    at one thread, and the other workloads (`legs`: name -> spec) likewise on
    smaller samples."""
    cores = host_cores()
    out = cpu_baseline_one(spec, cores, 20.0)
    out["cpu_model"] = cpu_model()
    out["single_thread"] = cpu_baseline_one(spec, 1, 60.0)
    out["other_workloads"] = {}
    for name, leg in legs.items():
        out["other_workloads"][name] = {
            "all_cores": cpu_baseline_one(leg, cores, 6.0),
            "single_thread": cpu_baseline_one(leg, 1, 6.0)}
    _omp_threads(cores)
    return out


def hbm_copy_probe(n_doubles: int = 2 ** 28, reps: int = 10):
    """Plain device-to-device copy of 2 GiB (torch's copy kernel) timed with
    HIP events: the HBM bandwidth a streaming kernel reaches on this GPU
    (bytes read + bytes written per second)."""
    import torch
    a = torch.empty(n_doubles, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    gbs = 2 * 8 * n_doubles / (ms * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return {"bytes_read": 8 * n_doubles, "bytes_written": 8 * n_doubles, "ms": ms, "GB/s": gbs,
            "frac_of_8TB/s": gbs / HBM_PEAK_GBS}


def bench_batched(n_systems, steps, seed=20260213):
    """256 independent LJ systems (N log-uniform in [64, 4096], P from
    {8, 16, 32, 64}, kT in [0.5, 1]) stepped together in one batch, against the
    same systems stepped one at a time with their own contexts."""
    import torch
    from paper_2602_13553_amd import pimd
    specs = inputs.batch_systems(n_systems=n_systems, seed=seed, nsteps=steps)
    work = sum(s.bead_atoms for s in specs) * steps
    b = pimd.Batch()
    ids = [b.add(s) for s in specs]
    for i, s in zip(ids, specs):
        b.set_state(i, s.x0, s.v0, 0)
    b.step(2)                       # plan, graph capture and first-touch outside the timing
    torch.cuda.synchronize()
    b.estimators(ids[0])
    t0 = time.perf_counter()
    b.step(steps)
    b.estimators(ids[0])            # waits for the batch stream
    tb = time.perf_counter() - t0
    b.close()
    # one at a time
    ctxs = []
    for s in specs:
        c = pimd.Context.from_spec(s, use_torch_workspace=False)
        c.set_state(s.x0, s.v0, 0)
        c.step(2)
        c.estimators()
        ctxs.append(c)
    t0 = time.perf_counter()
    for c in ctxs:
        c.step(steps)
        c.estimators()
    ts = time.perf_counter() - t0
    for c in ctxs:
        c.close()
    return {"workload": "%d LJ systems, N log-uniform [64,4096], P in {8,16,32,64}" % n_systems,
            "steps": steps, "bead_atoms": sum(s.bead_atoms for s in specs),
            "batched_bead_atom_steps_per_s": work / tb, "batched_s": tb,
            "one_at_a_time_bead_atom_steps_per_s": work / ts, "one_at_a_time_s": ts,
            "speedup": ts / tb}


def bench_external(steps=500, warmup=50):
    """External-force mode on the LJ liquid's shape (N=4000, P=32): the
    library's share of a step (positions out, forces in, one step), with the
    caller's force evaluation replaced by a fixed device array."""
    import dataclasses
    import torch
    from paper_2602_13553_amd import pimd
    lj = inputs.lj_liquid()
    spec = dataclasses.replace(lj, potential=pimd.PIMD_POT_EXTERNAL, box=(0.0, 0.0, 0.0))
    ctx = pimd.Context.from_spec(spec)
    ctx.set_state(spec.x0, spec.v0, 0)
    xd = torch.empty((spec.n_beads, spec.n_atoms, 3), dtype=torch.float64, device="cuda")
    fd = torch.zeros_like(xd)
    torch.cuda.synchronize()

    def one():
        ctx.get_positions(xd)
        ctx.set_forces(fd, 0.0)
        ctx.step(1)

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        one()
    ctx.get_positions(xd)
    ctx.set_forces(fd, 0.0)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    ctx.close()
    return {"workload": "external forces, N=4000, P=32 (library share: positions out, forces in, "
                        "one step; the caller's force evaluation excluded)",
            "ms_per_step": ms, "bead_atom_steps_per_s": spec.bead_atoms * 1e3 / ms,
            "steps": steps}


def bench_serving(n_jobs, seed=20260213):
    """Poisson arrivals at 20 jobs/s (harmonic, LJ or water-shaped; N
    log-uniform in [256, 32768]; P from {8..64}; 200-5000 steps), admitted under
    a 200 GB budget and stepped together, against one job at a time."""
    from paper_2602_13553_amd import serve
    tr = inputs.serving_trace(n_jobs=n_jobs, seed=seed)

    def progress(tag):
        state = {"last": 0}

        def f(done):
            if done >= state["last"] + 50 or done == n_jobs:
                state["last"] = done
                log("  %s: %d of %d jobs done" % (tag, done, n_jobs))
        return f

    rep = serve.serve(tr, hbm_budget=200e9, max_active=64, tick=32,
                      progress=progress("continuous batching")).summary()
    seq = serve.serve_sequential(tr, progress=progress("one at a time")).summary()
    offered = sum(j.n_atoms * j.n_beads * j.nsteps for j in tr) / max(tr[-1].arrival, 1e-9)
    return {"workload": "%d jobs, Poisson 20/s, harmonic/LJ/water, N in [256,32768], "
                        "P in {8,16,32,64}, 200-5000 steps" % n_jobs,
            "offered_bead_atom_steps_per_s": offered,
            "continuous_batching": rep, "one_at_a_time": seq}


def pair_roofline(workload, spec, x, avgs):
    """FP64 roofline of the force pass: 23 flops per ordered bead pair inside
    rc (LJ among the active atoms, counted on the final state), over the
    pass's average duration by HIP events.  The water-shaped system's bonds
    (2 per molecule, about 2% of the pairs' work) are not counted."""
    npairs = pairs_inside_cutoff(x, spec.box, spec.lj_rc, spec.lj_active)
    flops = LJ_FLOPS_PER_PAIR * npairs
    ach = flops / (avgs["pair"][0] * 1e-3) / 1e12
    # even P: the instantiation whose lanes take bead pairs
    kname = "k_pair<true>" if spec.n_beads % 2 == 0 else "k_pair<false>"
    return {"kernel": kname, "bound": "alu", "achieved": ach, "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": ach / FP64_PEAK_TFLOPS,
            "traffic": profiled_traffic(PROFILE_FILES.get((workload, "k_pair"), ""),
                                        _counter_name(kname)),
            "work_per_launch": "%d ordered bead pairs inside rc x %d flops" % (npairs, LJ_FLOPS_PER_PAIR),
            "launch_us": avgs["pair"][0] * 1e3}


def fused_kernel_name(spec, info):
    # the step passes are instantiated per splitting and fixcom
    tf = lambda v: "true" if v else "false"
    return (("k_fused_mfma<%d, %s, %s>" % (spec.n_beads, tf(spec.integrator), tf(spec.fixcom)))
            if info["transforms"] else "k_fused<%s>" % tf(spec.fixcom))


def fused_roofline(workload, spec, info, avgs):
    """HBM roofline of the step pass: the method's 120 B per bead*atom (read
    x, v~, f; write x, v~; 96 B with the trap's in-pass forces) over the
    pass's average duration by HIP events."""
    name = fused_kernel_name(spec, info)
    byts = (FUSED_BYTES_PAIR if spec.potential != inputs.POT_HARMONIC else FUSED_BYTES_EXT) * spec.bead_atoms
    ach = byts / (avgs["fused"][0] * 1e-3) / 1e9
    return {"kernel": name, "workload": spec.name, "bound": "hbm", "achieved": ach,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "traffic": profiled_traffic(PROFILE_FILES.get((workload, name), ""), _counter_name(name)),
            "bytes_per_launch": byts, "launch_us": avgs["fused"][0] * 1e3}


def leg(workload, steps, warmup, profile_steps, flags=0):
    """ms/step, throughput and per-kernel averages of one more workload."""
    title, make, _ = WORKLOADS[workload]
    spec = make()
    log("leg %s: %d warmup + %d timed steps" % (spec.name, warmup, steps))
    ms, est, prof, _, x, info = run_gpu(spec, steps, warmup, profile_steps, flags)
    avgs = kernel_avgs(prof)
    return spec, x, info, avgs, {"workload": title, "ms_per_step": ms,
                                 "bead_atom_steps_per_s": spec.bead_atoms * 1e3 / ms,
                                 "kernels_ms": {k: v[0] for k, v in avgs.items()},
                                 "launch": info}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--profile-steps", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-hbm-probe", action="store_true")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the P=32 and LJ legs")
    ap.add_argument("--batch-systems", type=int, default=256)
    ap.add_argument("--batch-steps", type=int, default=1000)
    ap.add_argument("--serve-jobs", type=int, default=100)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="water64",
                    help="workload of the timed steps (default: water-shaped, N=32766, P=64)")
    ap.add_argument("--transforms", choices=("auto", "valu"), default="auto",
                    help="valu: normal-mode transforms on the FP64 vector ALUs only")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    title, make, data = WORKLOADS[args.workload]
    spec = make()
    flags = 0
    if args.transforms == "valu":
        from paper_2602_13553_amd import pimd as _p
        flags = _p.PIMD_FLAG_VALU_TRANSFORMS
    log("workload %s: %d warmup + %d timed steps" % (spec.name, args.warmup, args.steps))
    ms_step, est, prof, ms_prof, x, info = run_gpu(spec, args.steps, args.warmup,
                                                   args.profile_steps, flags)
    ba = spec.bead_atoms
    value = ba * 1e3 / ms_step
    avgs = kernel_avgs(prof)
    log("ms/step %.4f (profiled %.4f); kernels %s" % (ms_step, ms_prof, avgs))

    # dominant kernel of the workload and its roofline
    dom = max(("fused", "pair"), key=lambda k: avgs[k][0] * avgs[k][1])
    if dom == "pair":
        roof = pair_roofline(args.workload, spec, x, avgs)
    else:
        roof = fused_roofline(args.workload, spec, info, avgs)

    out = {
        "metric": "ring-polymer bead*atom*steps/s",
        "value": value,
        "unit": "bead*atom*steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": data,
        "config": {"workload": title, "n_atoms": spec.n_atoms,
                   "n_beads": spec.n_beads, "bead_atoms": ba, "temp": spec.temp,
                   "hbar": spec.hbar, "rc": spec.lj_rc, "skin": spec.skin, "dt": spec.dt, "tau": spec.tau,
                   "ensemble": "NVT PILE-L", "integrator": "BAOAB",
                   "transforms": args.transforms},
        "roofline": roof,
        "step_pass_roofline": fused_roofline(args.workload, spec, info, avgs),
        "kernels_ms": {k: v[0] for k, v in avgs.items()},
        "launch": info,
        "estimators": {"kcv_per_atom": est["kcv"] / spec.n_atoms,
                       "kprim_per_atom": est["kprim"] / spec.n_atoms, "temp": est["temp"],
                       "pcv": est["pcv"], "ppr": est["ppr"], "pmd": est["pmd"]},
        "neighbor_lists": {"rlist": est["rlist"], "builds": est["n_rebuilds"],
                           "steps": args.warmup + args.profile_steps + args.steps},
    }
    legs_for_cpu = {}
    if not args.no_legs:
        for wl in ("water32", "lj"):
            if wl == args.workload:
                continue
            lspec, lx, linfo, lavgs, rec = leg(wl, 500, 50, 100)
            rec["pair_roofline"] = pair_roofline(wl, lspec, lx, lavgs)
            rec["step_pass_roofline"] = fused_roofline(wl, lspec, linfo, lavgs)
            out[wl] = rec
            legs_for_cpu[wl] = lspec
        legs_for_cpu["harmonic"] = inputs.harmonic_tiny()

    if not args.no_hbm_probe:
        # the step pass on a working set far beyond the 256 MB Infinity Cache:
        # the water-shaped system four times larger (8.4e6 bead*atoms; the
        # pass moves 120 B of algorithmic bytes per bead*atom, 1.0 GB)
        wspec, _, winfo, wavgs, rec = leg("water64x4", 30, 5, 30)
        rec["step_pass_roofline"] = fused_roofline("water64x4", wspec, winfo, wavgs)
        out["fused_roofline"] = rec["step_pass_roofline"]
        out["water64x4"] = rec
        from paper_2602_13553_amd import pimd as _p
        _, _, vinfo, vavgs, _ = leg("water64x4", 10, 3, 10, flags=_p.PIMD_FLAG_VALU_TRANSFORMS)
        out["water64x4"]["step_pass_valu_transforms"] = fused_roofline("water64x4", wspec, vinfo, vavgs)
        log("hbm copy probe")
        out["hbm_copy_probe"] = hbm_copy_probe()

    if not args.no_batch:
        ljt, ljmake, _ = WORKLOADS["lj"]
        log("OBABO splitting")
        ob = ljmake()
        ob.integrator = 1
        ms_ob, _, prof_ob, _, _, _ = run_gpu(ob, 500, 50, 100, flags)
        out["obabo"] = {"workload": ljt + ", OBABO splitting (two O half steps per step)",
                        "ms_per_step": ms_ob, "bead_atom_steps_per_s": ob.bead_atoms * 1e3 / ms_ob,
                        "kernels_ms": {k: v[0] for k, v in kernel_avgs(prof_ob).items()}}
        log("fixcom")
        fc = ljmake()
        fc.fixcom = 1
        ms_fc, _, prof_fc, _, _, _ = run_gpu(fc, 500, 50, 100, flags)
        out["fixcom"] = {"workload": ljt + ", fixcom (centroid COM velocity removed every step; "
                                           "the closing half-kick in a pass of its own)",
                         "ms_per_step": ms_fc, "bead_atom_steps_per_s": fc.bead_atoms * 1e3 / ms_fc,
                         "kernels_ms": {k: v[0] for k, v in kernel_avgs(prof_fc).items()}}
        log("NpT (BZP barostat)")
        out["npt"] = bench_npt(ljmake)
        log("bosonic exchange kernel")
        out["boson_spring"] = bench_boson()
        log("bosonic contexts")
        out["bosons"] = bench_bosons()
        log("external forces")
        out["external_forces"] = bench_external()
        log("batched: %d systems x %d steps" % (args.batch_systems, args.batch_steps))
        out["batched"] = bench_batched(args.batch_systems, args.batch_steps)
    if not args.no_serve:
        log("serving: %d jobs" % args.serve_jobs)
        out["serving"] = bench_serving(args.serve_jobs)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(spec, legs_for_cpu)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
