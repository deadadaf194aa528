"""Plain CPU FP64 oracle for the ring-polymer BAOAB + PILE-L step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(``paper_2602_13553_amd``) never imports it and shares no code with it.

The arithmetic lives in ``pimd_oracle.c`` (plain C, ``-O2 -ffp-contract=off``);
this module only marshals numpy arrays through ctypes.  Every array is FP64 in
the oracle's own layout ``[P][N][3]`` (bead, atom, Cartesian dim).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "pimd_oracle.c")

POT_NONE, POT_HARMONIC, POT_PAIR = 0, 1, 2


_SAN_PATH = os.path.join(_HERE, "liboracle_san.so")
# gcc flags of the sanitized build: address and undefined-behaviour checks,
# every finding fatal
SANITIZE_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                  "-fno-omit-frame-pointer", "-g"]


def build(force: bool = False, sanitize: bool = False) -> str:
    """Compile ``liboracle.so`` with gcc (OpenMP on, FMA contraction off);
    sanitize: ``liboracle_san.so`` with AddressSanitizer and
    UndefinedBehaviorSanitizer instead (same arithmetic flags).  The loader
    takes the library named by the environment variable ORACLE_LIB when it
    is set (the sanitized one needs its runtimes preloaded)."""
    path = _SAN_PATH if sanitize else _LIB_PATH
    if force or not os.path.exists(path) or (
        os.path.getmtime(path) < max(os.path.getmtime(_SRC),
                                     os.path.getmtime(os.path.join(_HERE, "pimd_oracle.h")))
    ):
        tmp = path + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-Wall"] + (SANITIZE_FLAGS if sanitize else []) + \
              ["-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, path)
    return path


class _System(C.Structure):
    _fields_ = [
        ("n_atoms", C.c_int32), ("n_beads", C.c_int32), ("nve", C.c_int32), ("pot", C.c_int32),
        ("temp", C.c_double), ("kB", C.c_double), ("hbar", C.c_double), ("mvv2e", C.c_double),
        ("dt", C.c_double), ("tau", C.c_double), ("tau_scale", C.c_double),
        ("box", C.c_double * 3), ("seed", C.c_uint64), ("omega", C.c_double),
        ("lj_eps", C.c_double), ("lj_sigma", C.c_double), ("lj_rc", C.c_double),
        ("bond_k", C.c_double), ("bond_r0", C.c_double),
        ("mass", C.POINTER(C.c_double)), ("lj_active", C.POINTER(C.c_int32)),
        ("n_bonds", C.c_int32), ("bonds", C.POINTER(C.c_int32)),
        ("atom_id", C.POINTER(C.c_int64)), ("integrator", C.c_int32), ("fixcom", C.c_int32),
        ("npt", C.c_int32), ("p_ext", C.c_double), ("tau_p", C.c_double),
        ("aniso", C.c_int32),
    ]


class _Baro(C.Structure):
    _fields_ = [("vw", C.c_double), ("box", C.c_double * 3), ("vwa", C.c_double * 3)]


class _Est(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("ekin", "espring", "epot", "etot", "kprim", "kcv", "temp",
                                          "pcv", "ppr", "pmd")]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(os.environ.get("ORACLE_LIB") or build())
        d = C.POINTER(C.c_double)
        u32 = C.POINTER(C.c_uint32)
        u64 = C.POINTER(C.c_uint64)
        S = C.POINTER(_System)
        sig = {
            "orc_nm_matrix": (None, [C.c_int32, d]),
            "orc_mode_lambda": (None, [C.c_int32, d]),
            "orc_to_normal": (None, [C.c_int32, C.c_int32, d, d]),
            "orc_from_normal": (None, [C.c_int32, C.c_int32, d, d]),
            "orc_philox4x32_10": (None, [u32, u32, u32]),
            "orc_gaussians": (None, [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64, d]),
            "orc_gaussians_q": (None, [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64,
                                       C.c_uint32, d]),
            "orc_free_rp_matrix": (None, [S, C.c_int32, C.c_double, d]),
            "orc_pile_coeffs": (None, [S, C.c_int32, d, d]),
            "orc_forces_bead": (C.c_double, [S, d, d]),
            "orc_forces": (None, [S, d, d, d]),
            "orc_virial_bead": (C.c_double, [S, d]),
            "orc_step": (None, [S, d, d, d, d, u64, C.c_int32]),
            "orc_step_positions": (None, [S, d, d, d, u64]),
            "orc_step_kick": (None, [S, d, d, C.c_uint64]),
            "orc_estimators": (None, [S, d, d, d, d, C.POINTER(_Est)]),
            "orc_spring_energy_nm": (C.c_double, [S, d]),
            "orc_kcv_nm": (C.c_double, [S, d, d]),
            "orc_baro_mass": (C.c_double, [S]),
            "orc_sinhc": (C.c_double, [C.c_double]),
            "orc_baro_kick": (None, [S, C.POINTER(_Baro), d, d, d, C.c_double]),
            "orc_baro_centroid_flow": (None, [C.c_double, C.c_double, d, d]),
            "orc_npt_step": (None, [S, C.POINTER(_Baro), d, d, d, d, u64, C.c_int32]),
            "orc_baro_energies": (None, [S, C.POINTER(_Baro), C.c_double, d]),
            "orc_virial_bead_diag": (None, [S, d, d]),
            "orc_boson_spring": (C.c_double, [C.c_int32, C.c_int32, C.c_double, C.c_double, d, d,
                                              d, d, d]),
            "orc_boson_forces": (C.c_double, [S, d, d, d]),
            "orc_boson_step": (None, [S, d, d, d, d, d, u64, C.c_int32]),
            "orc_boson_estimators": (None, [S, d, d, C.POINTER(_Est)]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(_lib, name)
            fn.restype = res
            fn.argtypes = args
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def nm_matrix(P: int) -> np.ndarray:
    M = np.zeros((P, P))
    lib().orc_nm_matrix(P, _dp(M))
    return M


def mode_lambda(P: int) -> np.ndarray:
    lam = np.zeros(P)
    lib().orc_mode_lambda(P, _dp(lam))
    return lam


def to_normal(a: np.ndarray) -> np.ndarray:
    P, N, _ = a.shape
    a = np.ascontiguousarray(a, dtype=np.float64)
    out = np.zeros_like(a)
    lib().orc_to_normal(P, N, _dp(a), _dp(out))
    return out


def from_normal(at: np.ndarray) -> np.ndarray:
    P, N, _ = at.shape
    at = np.ascontiguousarray(at, dtype=np.float64)
    out = np.zeros_like(at)
    lib().orc_from_normal(P, N, _dp(at), _dp(out))
    return out


def philox4x32_10(ctr, key) -> list[int]:
    c = (C.c_uint32 * 4)(*[int(v) & (2**32 - 1) for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & (2**32 - 1) for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def boson_spring(x: np.ndarray, kspring: float, beta_n: float, with_ev: bool = False, box=None):
    """Bosonic exchange spring energy V_B of bead positions x [P][N][3], its
    forces -dV_B/dx and the link probabilities [N][N] (l's last bead to l''s
    first); with_ev: also the weighted ring energy EV of the primitive
    estimator; box: periodic box lengths (links under the minimum image)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    P, N, _ = x.shape
    f = np.zeros_like(x)
    prob = np.zeros((N, N))
    ev = np.zeros(1)
    bx = None if box is None else np.ascontiguousarray(box, dtype=np.float64)
    v = lib().orc_boson_spring(N, P, kspring, beta_n, _dp(x), None if bx is None else _dp(bx),
                               _dp(f), _dp(prob), _dp(ev))
    return (v, f, prob, float(ev[0])) if with_ev else (v, f, prob)


def gaussians(seed: int, i: int, k: int, s: int, q: int = 0) -> np.ndarray:
    z = np.zeros(3)
    lib().orc_gaussians_q(seed, i, k, s, q, _dp(z))
    return z


@dataclass
class System:
    """Physical parameters of one ring-polymer system (oracle side)."""
    n_atoms: int
    n_beads: int
    mass: np.ndarray
    temp: float
    kB: float = 1.0
    hbar: float = 1.0
    mvv2e: float = 1.0
    dt: float = 0.01
    tau: float = 1.0
    tau_scale: float = 1.0
    nve: bool = False
    pot: int = POT_NONE
    box: tuple = (0.0, 0.0, 0.0)
    seed: int = 0
    omega: float = 0.0
    lj_eps: float = 0.0
    lj_sigma: float = 1.0
    lj_rc: float = 2.5
    bond_k: float = 0.0
    bond_r0: float = 0.0
    lj_active: np.ndarray | None = None
    bonds: np.ndarray | None = None
    atom_id: np.ndarray | None = None   # noise-counter index per atom (None: 0..N-1)
    integrator: int = 0                 # 0: BAOAB, 1: OBABO
    fixcom: int = 0                     # 1: centroid COM velocity removed every step
    npt: int = 0                        # 1: isotropic BZP barostat (OBABO only); nve -> NpH
    p_ext: float = 0.0                  # target pressure
    tau_p: float = 1.0                  # barostat time, W = 3 P N kB T tau_p^2
    aniso: int = 0                      # 1: anisotropic barostat (one v_W per dimension)
    _c: _System = field(default=None, init=False, repr=False)

    def cstruct(self) -> _System:
        self._mass = np.ascontiguousarray(self.mass, dtype=np.float64)
        s = _System()
        s.n_atoms, s.n_beads, s.nve, s.pot = self.n_atoms, self.n_beads, int(self.nve), self.pot
        s.temp, s.kB, s.hbar, s.mvv2e = self.temp, self.kB, self.hbar, self.mvv2e
        s.dt, s.tau, s.tau_scale = self.dt, self.tau, self.tau_scale
        s.box = (C.c_double * 3)(*self.box)
        s.seed = int(self.seed) & (2**64 - 1)
        s.omega = self.omega
        s.lj_eps, s.lj_sigma, s.lj_rc = self.lj_eps, self.lj_sigma, self.lj_rc
        s.bond_k, s.bond_r0 = self.bond_k, self.bond_r0
        s.integrator = int(self.integrator)
        s.fixcom = int(self.fixcom)
        s.npt, s.p_ext, s.tau_p = int(self.npt), float(self.p_ext), float(self.tau_p)
        s.aniso = int(self.aniso)
        s.mass = _dp(self._mass)
        if self.lj_active is not None:
            self._act = np.ascontiguousarray(self.lj_active, dtype=np.int32)
            s.lj_active = self._act.ctypes.data_as(C.POINTER(C.c_int32))
        if self.bonds is not None and len(self.bonds):
            self._bonds = np.ascontiguousarray(self.bonds, dtype=np.int32).reshape(-1, 2)
            s.n_bonds = self._bonds.shape[0]
            s.bonds = self._bonds.ctypes.data_as(C.POINTER(C.c_int32))
        if self.atom_id is not None:
            self._aid = np.ascontiguousarray(self.atom_id, dtype=np.int64)
            assert self._aid.shape == (self.n_atoms,)
            s.atom_id = self._aid.ctypes.data_as(C.POINTER(C.c_int64))
        self._c = s
        return s

    @classmethod
    def from_spec(cls, spec) -> "System":
        """Build from any object with the workload-spec attributes (duck-typed,
        so this package imports nothing from the product package)."""
        # 4: forces supplied by the caller (State.external); no built-in potential
        pot = {0: POT_NONE, 1: POT_HARMONIC, 2: POT_PAIR, 3: POT_PAIR, 4: POT_NONE}[int(spec.potential)]
        return cls(n_atoms=spec.n_atoms, n_beads=spec.n_beads, mass=np.asarray(spec.mass),
                   temp=spec.temp, kB=spec.kB, hbar=spec.hbar, mvv2e=spec.mvv2e, dt=spec.dt,
                   tau=spec.tau, tau_scale=spec.tau_scale, nve=bool(spec.ensemble in (1, 3)),
                   pot=pot, box=tuple(spec.box), seed=spec.seed, omega=spec.omega,
                   lj_eps=spec.lj_eps, lj_sigma=spec.lj_sigma, lj_rc=spec.lj_rc,
                   bond_k=spec.bond_k, bond_r0=spec.bond_r0, lj_active=spec.lj_active,
                   bonds=spec.bonds, integrator=int(getattr(spec, "integrator", 0)),
                   fixcom=int(getattr(spec, "fixcom", 0)),
                   npt=int(spec.ensemble in (2, 3)), p_ext=float(getattr(spec, "p_ext", 0.0)),
                   tau_p=float(getattr(spec, "tau_p", 1.0)),
                   aniso=int(getattr(spec, "baro_aniso", 0)))

    # --- per-function wrappers -------------------------------------------
    def free_rp_matrix(self, k: int, h: float) -> np.ndarray:
        A = np.zeros(4)
        lib().orc_free_rp_matrix(C.byref(self.cstruct()), k, h, _dp(A))
        return A.reshape(2, 2)

    def pile_coeffs(self, k: int) -> tuple[float, float]:
        c1, c2 = C.c_double(), C.c_double()
        lib().orc_pile_coeffs(C.byref(self.cstruct()), k, C.byref(c1), C.byref(c2))
        return c1.value, c2.value

    def forces(self, x: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
        x = np.ascontiguousarray(x, dtype=np.float64)
        if x.shape != (self.n_beads, self.n_atoms, 3):
            raise ValueError("x must be [n_beads][n_atoms][3], got %s" % (x.shape,))
        f = np.zeros_like(x)
        U = np.zeros(self.n_beads)
        lib().orc_forces(C.byref(self.cstruct()), _dp(x), _dp(f), _dp(U))
        return f, U

    def virial(self, xk: np.ndarray) -> float:
        """Cell virial Tr Xi of one bead configuration xk [N][3]."""
        xk = np.ascontiguousarray(xk, dtype=np.float64)
        if xk.shape != (self.n_atoms, 3):
            raise ValueError("xk must be [n_atoms][3], got %s" % (xk.shape,))
        return lib().orc_virial_bead(C.byref(self.cstruct()), _dp(xk))

    def virial_diag(self, xk: np.ndarray) -> np.ndarray:
        """Diagonal (Xi_xx, Xi_yy, Xi_zz) of one bead's cell virial tensor."""
        xk = np.ascontiguousarray(xk, dtype=np.float64)
        if xk.shape != (self.n_atoms, 3):
            raise ValueError("xk must be [n_atoms][3], got %s" % (xk.shape,))
        w = np.zeros(3)
        lib().orc_virial_bead_diag(C.byref(self.cstruct()), _dp(xk), _dp(w))
        return w

    def spring_energy_nm(self, x: np.ndarray) -> float:
        x = np.ascontiguousarray(x, dtype=np.float64)
        return lib().orc_spring_energy_nm(C.byref(self.cstruct()), _dp(x))

    def kcv_nm(self, x: np.ndarray, f: np.ndarray) -> float:
        x = np.ascontiguousarray(x, dtype=np.float64)
        f = np.ascontiguousarray(f, dtype=np.float64)
        return lib().orc_kcv_nm(C.byref(self.cstruct()), _dp(x), _dp(f))


ESTIMATOR_NAMES = ("ekin", "espring", "epot", "etot", "kprim", "kcv", "temp", "pcv", "ppr", "pmd")


class State:
    """Oracle integrator state: Cartesian x, normal-mode v~, forces f, step s."""

    @classmethod
    def from_spec(cls, spec, step: int = 0) -> "State":
        return cls(System.from_spec(spec), spec.x0, spec.v0, step)

    def __init__(self, system: System, x: np.ndarray, v: np.ndarray, step: int = 0):
        self.sys = system
        self.x = np.ascontiguousarray(x, dtype=np.float64).copy()
        self.vt = to_normal(np.ascontiguousarray(v, dtype=np.float64))
        self.f, self.U = system.forces(self.x)
        self.step_count = np.array([step], dtype=np.uint64)
        if system.npt:
            self.baro = _Baro()
            self.baro.vw = 0.0
            self.baro.box = (C.c_double * 3)(*system.box)
            self.baro.vwa = (C.c_double * 3)(0.0, 0.0, 0.0)

    @property
    def box(self) -> tuple:
        return tuple(self.baro.box) if self.sys.npt else tuple(self.sys.box)

    def _cs(self) -> _System:
        """The system's struct with the current box."""
        s = self.sys.cstruct()
        if self.sys.npt:
            s.box = (C.c_double * 3)(*self.baro.box)
        return s

    @property
    def v(self) -> np.ndarray:
        """Cartesian bead velocities M^T v~."""
        return from_normal(self.vt)

    @property
    def p(self) -> np.ndarray:
        return self.v * self.sys.mass[None, :, None]

    def step(self, n: int = 1) -> None:
        s = self.sys.cstruct()
        if self.sys.npt:
            lib().orc_npt_step(C.byref(s), C.byref(self.baro), _dp(self.x), _dp(self.vt),
                               _dp(self.f), _dp(self.U),
                               self.step_count.ctypes.data_as(C.POINTER(C.c_uint64)), int(n))
            return
        lib().orc_step(C.byref(s), _dp(self.x), _dp(self.vt), _dp(self.f), _dp(self.U),
                       self.step_count.ctypes.data_as(C.POINTER(C.c_uint64)), int(n))

    def baro_energies(self) -> dict:
        """NpT: volume, K_W, U_W, J_W and the enthalpy of App. A, and v_W."""
        out = np.zeros(5)
        lib().orc_baro_energies(C.byref(self._cs()), C.byref(self.baro),
                                self.estimators()["etot"], _dp(out))
        vw = tuple(self.baro.vwa) if self.sys.aniso else self.baro.vw
        return dict(zip(("volume", "kw", "uw", "jw", "enthalpy"), out.tolist()), vw=vw)

    # --- forces supplied by the caller (an external potential) -----------
    @classmethod
    def external(cls, system: System, x: np.ndarray, v: np.ndarray, force_fn, step: int = 0) -> "State":
        """A state whose forces come from ``force_fn(x) -> (f [P][N][3], U [P])``
        (per-bead forces and energies) instead of the built-in potential."""
        st = cls(system, x, v, step)
        st._set_forces(force_fn)
        return st

    def _set_forces(self, force_fn) -> None:
        f, U = force_fn(self.x.copy())
        self.f = np.ascontiguousarray(f, dtype=np.float64).copy()
        self.U = np.ascontiguousarray(U, dtype=np.float64).reshape(self.sys.n_beads).copy()

    def step_external(self, force_fn, n: int = 1) -> None:
        """n steps, each B A O A (orc_step_positions), the caller's forces at
        the new positions, then the closing B (orc_step_kick): the step of
        ``step`` with the force call made by ``force_fn``."""
        s = self.sys.cstruct()
        for _ in range(int(n)):
            lib().orc_step_positions(C.byref(s), _dp(self.x), _dp(self.vt), _dp(self.f),
                                     self.step_count.ctypes.data_as(C.POINTER(C.c_uint64)))
            self._set_forces(force_fn)
            lib().orc_step_kick(C.byref(s), _dp(self.vt), _dp(self.f), int(self.step_count[0]) - 1)

    def estimators(self) -> dict:
        e = _Est()
        lib().orc_estimators(C.byref(self._cs()), _dp(self.x), _dp(self.vt), _dp(self.f),
                             _dp(self.U), C.byref(e))
        return {n: getattr(e, n) for n in ESTIMATOR_NAMES}


class BosonState:
    """Bosonic ring polymers in Cartesian coordinates (the bosonic fix's
    step): positions x and bead velocities v [P][N][3], total forces f."""

    def __init__(self, system: System, x: np.ndarray, v: np.ndarray, step: int = 0):
        if len(set(np.asarray(system.mass).tolist())) != 1:
            raise ValueError("bosons of one species: all masses equal")
        self.sys = system
        self.x = np.ascontiguousarray(x, dtype=np.float64).copy()
        self.v = np.ascontiguousarray(v, dtype=np.float64).copy()
        self.f = np.zeros_like(self.x)
        self.U = np.zeros(system.n_beads)
        self.vb = np.zeros(1)
        self.vb[0] = lib().orc_boson_forces(C.byref(system.cstruct()), _dp(self.x), _dp(self.f),
                                            _dp(self.U))
        self.step_count = np.array([step], dtype=np.uint64)

    def step(self, n: int = 1) -> None:
        lib().orc_boson_step(C.byref(self.sys.cstruct()), _dp(self.x), _dp(self.v), _dp(self.f),
                             _dp(self.U), _dp(self.vb),
                             self.step_count.ctypes.data_as(C.POINTER(C.c_uint64)), int(n))

    @classmethod
    def from_spec(cls, spec, step: int = 0) -> "BosonState":
        return cls(System.from_spec(spec), spec.x0, spec.v0, step)

    def estimators(self) -> dict:
        """App. A's bosonic outputs at the current (synchronized) state:
        ekin, espring (V_B), epot, etot, kprim (bosonic K_PR), kcv (holds
        K_VR, the virial estimator), temp; pressures 0."""
        e = _Est()
        lib().orc_boson_estimators(C.byref(self.sys.cstruct()), _dp(self.x), _dp(self.v),
                                   C.byref(e))
        return {n: getattr(e, n) for n in ESTIMATOR_NAMES}

    @property
    def p(self) -> np.ndarray:
        """Cartesian bead momenta m v."""
        return np.asarray(self.sys.mass)[None, :, None] * self.v

    def energies(self) -> dict:
        """K (Cartesian), the exchange spring energy V_B, U, H = K + V_B + U."""
        m = np.asarray(self.sys.mass)[None, :, None]
        k = float((0.5 * m * self.sys.mvv2e * self.v * self.v).sum())
        u = float(self.U.sum())
        return {"ekin": k, "vb": float(self.vb[0]), "epot": u, "etot": k + float(self.vb[0]) + u}
