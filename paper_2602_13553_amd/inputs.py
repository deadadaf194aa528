"""Seeded synthetic workloads for the ring-polymer PIMD step.

This module builds inputs only: lattices, water geometry, masses, parameters
and Maxwell-Boltzmann velocity draws.  It holds none of the integrator's
arithmetic (no normal modes, no propagation, no thermostat, no forces), so that
the GPU library and the CPU oracle can both be fed from it.

Every generator takes a seed and uses numpy's PCG64 stream; the same seed gives
the same arrays everywhere.  Arrays are FP64 in the host layout ``[P][N][3]``
(bead, atom, Cartesian dim).

Workloads (shapes of the paper's water benchmarks and of the reduced-unit
test systems it motivates):

* ``harmonic_tiny``   N=64, P=4 distinguishable particles in a harmonic trap
                      (m = omega = hbar = 1, kT = 0.25, dt = 0.05, tau = 1).
* ``lj_liquid``       LJ quantum liquid, FCC start at reduced density 0.8,
                      kT = 0.7, hbar = 0.1, rc = 2.5, P = 32, dt = 0.002, tau = 0.5.
* ``water``           water-shaped: O-H harmonic bonds plus O-O LJ at 9 A,
                      1 g/cm^3, 300 K, real units (kcal/mol, A, fs, amu).
* ``batch_systems``   256 independent LJ systems, N log-uniform in [64, 4096],
                      P from {8, 16, 32, 64}, kT uniform in [0.5, 1.0].
* ``serving_trace``   Poisson job arrivals mixing the three kinds above.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

# --- physical constants (CODATA 2018, exact SI definitions) ------------------
_HBAR_SI = 1.054571817e-34       # J s
_KB_SI = 1.380649e-23            # J / K
_NA = 6.02214076e23              # 1 / mol
_AMU = 1.66053906660e-27         # kg
_KCAL = 4184.0                   # J

#: real units: energy kcal/mol, length Angstrom, time fs, mass amu
REAL_KB = _KB_SI * _NA / _KCAL                    # kcal/mol/K
REAL_HBAR = _HBAR_SI * _NA / _KCAL * 1e15         # kcal/mol * fs
REAL_MVV2E = _AMU * 1e10 * _NA / _KCAL            # kcal/mol per amu (A/fs)^2

POT_NONE, POT_HARMONIC, POT_LJ, POT_WATER = 0, 1, 2, 3
NVT, NVE, NPT, NPH = 0, 1, 2, 3


@dataclass
class SystemSpec:
    """One ring-polymer system: parameters, topology and initial state."""
    name: str
    n_atoms: int
    n_beads: int
    temp: float
    kB: float
    hbar: float
    mvv2e: float
    dt: float
    tau: float
    tau_scale: float
    ensemble: int
    box: tuple
    seed: int
    potential: int
    mass: np.ndarray
    x0: np.ndarray                  # [P][N][3] Cartesian bead positions
    v0: np.ndarray                  # [P][N][3] Cartesian bead velocities
    omega: float = 0.0              # harmonic trap
    lj_eps: float = 0.0
    lj_sigma: float = 1.0
    lj_rc: float = 2.5
    bond_k: float = 0.0
    bond_r0: float = 0.0
    skin: float = 0.3               # neighbor-list skin (GPU library only)
    integrator: int = 0             # 0: BAOAB, 1: OBABO
    fixcom: int = 0                 # 1: remove the centroids' COM velocity every step
    p_ext: float = 0.0              # NPT, NPH: target pressure
    tau_p: float = 1.0              # NPT, NPH: barostat time
    lj_active: np.ndarray | None = None   # [N] 0/1
    bonds: np.ndarray | None = None       # [n_bonds][2]
    nsteps: int = 0                 # length of the workload's run
    bosonic: int = 0                # 1: identical bosons with exchange (Cartesian beads)
    baro_aniso: int = 0             # NPT, NPH: 1 = one barostat velocity per dimension
    extra: dict = field(default_factory=dict)

    @property
    def bead_atoms(self) -> int:
        return self.n_atoms * self.n_beads

    def with_beads(self, P: int, seed: int | None = None) -> "SystemSpec":
        """Same physical system with P beads and freshly drawn bead states."""
        rng = np.random.default_rng(self.seed if seed is None else seed)
        x1 = self.x0.mean(axis=0)
        jit = self.extra.get("bead_jitter", 0.0)
        x0 = x1[None] + jit * rng.standard_normal((P,) + x1.shape)
        v0 = _mb_velocities(rng, P, self.mass, self.temp * self.kB, self.mvv2e)
        return replace(self, n_beads=P, x0=x0, v0=v0)


def _mb_velocities(rng, P, mass, kT, mvv2e):
    """Cartesian bead velocities at the ring-polymer temperature P*T."""
    sd = np.sqrt(P * kT / (mass * mvv2e))
    return rng.standard_normal((P, mass.shape[0], 3)) * sd[None, :, None]


def fcc_sites(n_cells: int, a: float) -> np.ndarray:
    base = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    g = np.arange(n_cells)
    cells = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    return ((cells[:, None, :] + base[None, :, :]).reshape(-1, 3) * a).astype(np.float64)


# --- harmonic trap (config: N=64, P=4) ------------------------------------------
def harmonic_tiny(seed: int = 20260213, n_atoms: int = 64, n_beads: int = 4,
                  nsteps: int = 2000, ensemble: int = NVT) -> SystemSpec:
    rng = np.random.default_rng(seed)
    kT, m = 0.25, 1.0
    mass = np.full(n_atoms, m)
    x0 = 0.1 * rng.standard_normal((n_beads, n_atoms, 3))
    v0 = _mb_velocities(rng, n_beads, mass, kT, 1.0)
    return SystemSpec(name="harmonic N=%d P=%d" % (n_atoms, n_beads), n_atoms=n_atoms,
                      n_beads=n_beads, temp=kT, kB=1.0, hbar=1.0, mvv2e=1.0, dt=0.05, tau=1.0,
                      tau_scale=1.0, ensemble=ensemble, box=(0.0, 0.0, 0.0), seed=seed,
                      potential=POT_HARMONIC, mass=mass, x0=x0, v0=v0, omega=1.0, nsteps=nsteps)


def free_ring_polymer(seed: int = 7, n_atoms: int = 16, n_beads: int = 8, kT: float = 1.0,
                      hbar: float = 1.0, dt: float = 0.01, ensemble: int = NVE) -> SystemSpec:
    """Non-interacting ring polymers (U = 0), for conservation tests."""
    rng = np.random.default_rng(seed)
    mass = rng.uniform(1.0, 4.0, n_atoms)
    x0 = 0.2 * rng.standard_normal((n_beads, n_atoms, 3))
    v0 = _mb_velocities(rng, n_beads, mass, kT, 1.0)
    return SystemSpec(name="free RP", n_atoms=n_atoms, n_beads=n_beads, temp=kT, kB=1.0,
                      hbar=hbar, mvv2e=1.0, dt=dt, tau=1.0, tau_scale=1.0, ensemble=ensemble,
                      box=(0.0, 0.0, 0.0), seed=seed, potential=POT_NONE, mass=mass, x0=x0, v0=v0)


def cartesian_tau(n_beads: int, kT: float, hbar: float) -> float:
    """App. D's default damping time of the Cartesian thermostat, 1/(2 omega_n)
    with omega_n = P kB T / hbar."""
    return hbar / (2.0 * n_beads * kT)


def trapped_bosons(n_atoms: int = 16, n_beads: int = 8, kT: float = 0.5, hbar: float = 1.0,
                   omega: float = 1.0, dt: float = 0.02, seed: int = 20260213,
                   spread: float = 0.8, ensemble: int = NVT, integrator: int = 0) -> SystemSpec:
    """Identical bosons (m = 1) in a harmonic trap, reduced units, with the
    Cartesian thermostat's default damping time: centers N(0, spread^2), bead
    offsets N(0, 0.1^2), Maxwell-Boltzmann bead velocities at P*T."""
    rng = np.random.default_rng(seed)
    mass = np.ones(n_atoms)
    x0 = spread * rng.standard_normal((1, n_atoms, 3)) + 0.1 * rng.standard_normal((n_beads, n_atoms, 3))
    v0 = _mb_velocities(rng, n_beads, mass, kT, 1.0)
    return SystemSpec(name="bosons trap N=%d P=%d" % (n_atoms, n_beads), n_atoms=n_atoms,
                      n_beads=n_beads, temp=kT, kB=1.0, hbar=hbar, mvv2e=1.0, dt=dt,
                      tau=cartesian_tau(n_beads, kT, hbar), tau_scale=1.0, ensemble=ensemble,
                      box=(0.0, 0.0, 0.0), seed=seed, potential=POT_HARMONIC, mass=mass, x0=x0,
                      v0=v0, omega=omega, integrator=integrator, bosonic=1)


# --- Lennard-Jones quantum liquid ------------------------------------------------
def lj_liquid(n_atoms: int = 4000, n_beads: int = 32, rho: float = 0.8, kT: float = 0.7,
              hbar: float = 0.1, dt: float = 0.002, tau: float = 0.5, rc: float = 2.5,
              seed: int = 20260213, jitter: float = 0.01, nsteps: int = 1000,
              ensemble: int = NVT, skin: float = 0.2) -> SystemSpec:
    """FCC start (first n_atoms sites of the smallest cubic FCC block that holds
    them), cubic box L = (N/rho)^(1/3), independent N(0, jitter^2) offsets per
    (bead, atom, dim)."""
    rng = np.random.default_rng(seed)
    L = (n_atoms / rho) ** (1.0 / 3.0)
    nc = max(1, math.ceil((n_atoms / 4.0) ** (1.0 / 3.0) - 1e-9))
    sites = fcc_sites(nc, L / nc)[:n_atoms]
    mass = np.ones(n_atoms)
    x0 = sites[None] + jitter * rng.standard_normal((n_beads, n_atoms, 3))
    v0 = _mb_velocities(rng, n_beads, mass, kT, 1.0)
    return SystemSpec(name="LJ N=%d P=%d" % (n_atoms, n_beads), n_atoms=n_atoms,
                      n_beads=n_beads, temp=kT, kB=1.0, hbar=hbar, mvv2e=1.0, dt=dt, tau=tau,
                      tau_scale=1.0, ensemble=ensemble, box=(L, L, L), seed=seed,
                      potential=POT_LJ, mass=mass, x0=x0, v0=v0, lj_eps=1.0, lj_sigma=1.0,
                      lj_rc=rc, skin=skin, nsteps=nsteps,
                      extra={"rho": rho, "bead_jitter": jitter})


def lj_bosons(n_atoms: int = 108, n_beads: int = 8, rho: float = 0.8, kT: float = 1.0,
              hbar: float = 0.5, dt: float = 0.002, seed: int = 20260213, skin: float = 0.2,
              ensemble: int = NVT, integrator: int = 0) -> SystemSpec:
    """An LJ liquid of identical bosons (a helium-like quantum liquid in
    reduced units: thermal wavelength sqrt(2 pi hbar^2/(m kT)) = 1.25 sigma at
    the defaults, above the spacing at rho = 0.8), FCC start, the Cartesian
    thermostat's default damping time."""
    s = lj_liquid(n_atoms=n_atoms, n_beads=n_beads, rho=rho, kT=kT, hbar=hbar, dt=dt,
                  tau=cartesian_tau(n_beads, kT, hbar), seed=seed, ensemble=ensemble, skin=skin)
    return replace(s, name="LJ bosons N=%d P=%d" % (n_atoms, n_beads), integrator=integrator,
                   bosonic=1)


# --- water-shaped system ----------------------------------------------------------
def water(n_atoms: int = 32768, n_beads: int = 32, seed: int = 20260213, temp: float = 300.0,
          dt: float = 0.25, tau: float = 100.0, density: float = 1.0, nsteps: int = 500,
          ensemble: int = NVT, skin: float = 0.3, jitter: float = 0.01) -> SystemSpec:
    """Water-shaped system in real units.  n_atoms is rounded down to whole
    molecules (32768 -> 10922 molecules, 32766 atoms).  O atoms sit on the first
    n_mol sites of the smallest cubic grid that holds them; each molecule gets
    two H at r0 = 0.96 A with a 104.52 degree H-O-H angle in a random
    orientation.  Atom order: O, H, H per molecule."""
    rng = np.random.default_rng(seed)
    n_mol = n_atoms // 3
    N = 3 * n_mol
    mO, mH = 15.999, 1.008
    mass_g = n_mol * (mO + 2 * mH) * _AMU * 1e3
    L = (mass_g / density * 1e24) ** (1.0 / 3.0)
    ng = math.ceil(n_mol ** (1.0 / 3.0) - 1e-9)
    g = np.arange(ng)
    grid = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)[:n_mol]
    O = (grid + 0.5) * (L / ng)
    r0, ang = 0.96, math.radians(104.52)
    # random orthonormal frames from normalized Gaussian quaternions
    q = rng.standard_normal((n_mol, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, xq, yq, zq = q.T
    R = np.stack([
        np.stack([1 - 2 * (yq * yq + zq * zq), 2 * (xq * yq - zq * w), 2 * (xq * zq + yq * w)], -1),
        np.stack([2 * (xq * yq + zq * w), 1 - 2 * (xq * xq + zq * zq), 2 * (yq * zq - xq * w)], -1),
        np.stack([2 * (xq * zq - yq * w), 2 * (yq * zq + xq * w), 1 - 2 * (xq * xq + yq * yq)], -1),
    ], axis=1)
    h1 = np.array([r0 * math.sin(ang / 2), 0.0, r0 * math.cos(ang / 2)])
    h2 = np.array([-r0 * math.sin(ang / 2), 0.0, r0 * math.cos(ang / 2)])
    H1 = O + R @ h1
    H2 = O + R @ h2
    pos = np.stack([O, H1, H2], axis=1).reshape(N, 3)
    mass = np.tile([mO, mH, mH], n_mol).astype(np.float64)
    lj_active = np.tile([1, 0, 0], n_mol).astype(np.int32)
    base = 3 * np.arange(n_mol)
    bonds = np.concatenate([np.stack([base, base + 1], 1), np.stack([base, base + 2], 1)])
    bonds = bonds[np.lexsort((bonds[:, 1], bonds[:, 0]))].astype(np.int32)
    kT = REAL_KB * temp
    x0 = pos[None] + jitter * rng.standard_normal((n_beads, N, 3))
    v0 = _mb_velocities(rng, n_beads, mass, kT, REAL_MVV2E)
    return SystemSpec(name="water N=%d P=%d" % (N, n_beads), n_atoms=N, n_beads=n_beads,
                      temp=temp, kB=REAL_KB, hbar=REAL_HBAR, mvv2e=REAL_MVV2E, dt=dt, tau=tau,
                      tau_scale=1.0, ensemble=ensemble, box=(L, L, L), seed=seed,
                      potential=POT_WATER, mass=mass, x0=x0, v0=v0, lj_eps=0.155,
                      lj_sigma=3.165, lj_rc=9.0, bond_k=450.0, bond_r0=0.96, skin=skin,
                      lj_active=lj_active, bonds=bonds, nsteps=nsteps,
                      extra={"n_mol": n_mol, "bead_jitter": jitter})


# --- many independent systems --------------------------------------------------------
def batch_systems(n_systems: int = 256, seed: int = 20260213, n_min: int = 64,
                  n_max: int = 4096, beads=(8, 16, 32, 64), kT_range=(0.5, 1.0),
                  nsteps: int = 1000) -> list[SystemSpec]:
    """Independent LJ systems (physics of ``lj_liquid``): N log-uniform in
    [n_min, n_max], P uniform over ``beads``, kT uniform in ``kT_range``."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(n_systems):
        N = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        P = int(rng.choice(beads))
        kT = float(rng.uniform(*kT_range))
        spec = lj_liquid(n_atoms=N, n_beads=P, kT=kT, seed=seed * 1000003 + s, nsteps=nsteps)
        spec.name = "batch[%d] LJ N=%d P=%d" % (s, N, P)
        out.append(spec)
    return out


@dataclass
class Job:
    job_id: int
    arrival: float          # seconds after the start of the trace
    kind: str               # "harmonic" | "lj" | "water"
    n_atoms: int
    n_beads: int
    nsteps: int
    seed: int

    def spec(self) -> SystemSpec:
        if self.kind == "harmonic":
            s = harmonic_tiny(seed=self.seed, n_atoms=self.n_atoms, n_beads=self.n_beads,
                              nsteps=self.nsteps)
        elif self.kind == "lj":
            s = lj_liquid(n_atoms=self.n_atoms, n_beads=self.n_beads, seed=self.seed,
                          nsteps=self.nsteps)
        else:
            s = water(n_atoms=self.n_atoms, n_beads=self.n_beads, seed=self.seed,
                      nsteps=self.nsteps)
        s.name = "job%d %s" % (self.job_id, s.name)
        return s


def serving_trace(n_jobs: int = 600, rate: float = 20.0, seed: int = 20260213,
                  n_range=(256, 32768), beads=(8, 16, 32, 64), steps_range=(200, 5000),
                  kinds=("harmonic", "lj", "water")) -> list[Job]:
    """Poisson arrivals at ``rate`` jobs/s; kind uniform over ``kinds``; N
    log-uniform in ``n_range`` (whole molecules for water); P uniform over
    ``beads``; nsteps uniform in ``steps_range``."""
    rng = np.random.default_rng(seed)
    t = 0.0
    jobs = []
    for j in range(n_jobs):
        t += rng.exponential(1.0 / rate)
        kind = str(rng.choice(kinds))
        N = int(round(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))))
        if kind == "water":
            N = max(3, 3 * (N // 3))
        P = int(rng.choice(beads))
        ns = int(rng.integers(steps_range[0], steps_range[1] + 1))
        jobs.append(Job(j, t, kind, N, P, ns, seed * 7919 + j))
    return jobs
