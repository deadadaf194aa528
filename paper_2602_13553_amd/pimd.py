"""Python binding of ``libpimd.so`` (C ABI in ``include/pimd.h``).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  PyTorch supplies the device workspace (``torch.empty`` on ``cuda``)
so that device memory is accounted by torch's allocator.  If the library is
missing, every entry point raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpimd.so")

PIMD_OK = 0
ERRORS = {-1: "PIMD_ERR_ARG", -2: "PIMD_ERR_OOM", -3: "PIMD_ERR_DEVICE", -4: "PIMD_ERR_STATE",
          -5: "PIMD_ERR_NONFINITE", -6: "PIMD_ERR_UNSUPPORTED", -7: "PIMD_ERR_OVERFLOW"}
PIMD_ERR_ARG, PIMD_ERR_OOM, PIMD_ERR_DEVICE, PIMD_ERR_STATE = -1, -2, -3, -4
PIMD_ERR_NONFINITE, PIMD_ERR_UNSUPPORTED, PIMD_ERR_OVERFLOW = -5, -6, -7
PIMD_NVT, PIMD_NVE, PIMD_NPT, PIMD_NPH = 0, 1, 2, 3
PIMD_BAOAB, PIMD_OBABO = 0, 1
PIMD_POT_NONE, PIMD_POT_HARMONIC, PIMD_POT_LJ, PIMD_POT_WATER, PIMD_POT_EXTERNAL = 0, 1, 2, 3, 4
PIMD_FLAG_VALU_TRANSFORMS = 1
PIMD_FLAG_MFMA_TRANSFORMS = 2
PIMD_FLAG_CLUSTER_PAIRS = 4
PIMD_FLAG_ATOM_PAIRS = 8
PIMD_FLAG_NO_GRAPHS = 16
PIMD_PAIR_SUBGROUPS_SHIFT = 8


def PIMD_PAIR_SUBGROUPS(S: int) -> int:
    """Flag bits that fix the force pass's lane sub-groups per atom (S in 1..16)."""
    code = {1: 1, 2: 2, 4: 3, 8: 4, 16: 5}[S]
    return code << PIMD_PAIR_SUBGROUPS_SHIFT
ESTIMATOR_NAMES = ("ekin", "espring", "epot", "etot", "kprim", "kcv", "temp", "pcv", "ppr", "pmd")
NEST = len(ESTIMATOR_NAMES)   # PIMD_NEST
EXPORTED = ("pimd_workspace_bytes", "pimd_create", "pimd_set_state", "pimd_step",
            "pimd_get_estimators", "pimd_get_state", "pimd_get_barostat", "pimd_set_barostat",
            "pimd_boson_spring", "pimd_boson_spring_noalloc",
            "pimd_reset_averages",
            "pimd_get_positions",
            "pimd_set_forces", "pimd_destroy",
            "pimd_last_error", "pimd_profile_begin", "pimd_profile_end", "pimd_get_launch_info",
            "pimd_batch_create", "pimd_batch_add", "pimd_batch_remove", "pimd_batch_set_state",
            "pimd_batch_set_budget", "pimd_batch_step", "pimd_batch_get_estimators",
            "pimd_batch_get_state", "pimd_batch_destroy", "pimd_batch_last_error")
KERNEL_NAMES = ("fused", "pair", "close", "finalize")


class PimdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "PIMD_ERR"), code, msg))
        self.code = code


class pimd_params(C.Structure):
    _fields_ = [
        ("n_atoms", C.c_int32), ("n_beads", C.c_int32), ("ensemble", C.c_int32),
        ("potential", C.c_int32), ("temp", C.c_double), ("kB", C.c_double), ("hbar", C.c_double),
        ("mvv2e", C.c_double), ("dt", C.c_double), ("tau", C.c_double), ("tau_scale", C.c_double),
        ("box", C.c_double * 3), ("seed", C.c_uint64), ("omega", C.c_double),
        ("lj_eps", C.c_double), ("lj_sigma", C.c_double), ("lj_rc", C.c_double),
        ("skin", C.c_double), ("bond_k", C.c_double), ("bond_r0", C.c_double),
        ("nbr_capacity", C.c_int32), ("flags", C.c_int32), ("integrator", C.c_int32),
        ("fixcom", C.c_int32), ("p_ext", C.c_double), ("tau_p", C.c_double),
        ("bosonic", C.c_int32), ("baro_aniso", C.c_int32),
    ]


class pimd_topology(C.Structure):
    _fields_ = [("lj_active", C.POINTER(C.c_int32)), ("n_bonds", C.c_int32),
                ("bonds", C.POINTER(C.c_int32))]


class pimd_estimators(C.Structure):
    _fields_ = [("step", C.c_uint64), ("value", C.c_double * NEST), ("count", C.c_uint64),
                ("sum", C.c_double * NEST), ("sumsq", C.c_double * NEST), ("nonfinite", C.c_int32),
                ("overflow", C.c_int32), ("n_rebuilds", C.c_uint64), ("rlist", C.c_double),
                ("volume", C.c_double), ("vw", C.c_double), ("enthalpy", C.c_double),
                ("vwa", C.c_double * 3)]


class pimd_profile(C.Structure):
    _fields_ = [("launches", C.c_uint64 * 4), ("ms", C.c_double * 4)]


class pimd_launch_info(C.Structure):
    _fields_ = [("transforms", C.c_int32), ("fused_blocks", C.c_int32),
                ("pair_subgroups", C.c_int32), ("pair_blocks", C.c_int32), ("cells", C.c_int32),
                ("cluster_pairs", C.c_int32), ("bead_pairs", C.c_int32)]


_lib = None


def load() -> C.CDLL:
    """Load libpimd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libpimd.so is not built (run __graft_entry__.build())")
        # torch ships its own HIP runtime under the same soname
        # (libamdhip64.so.7); loading torch first makes libpimd.so bind to that
        # one, so the process holds a single HIP/HSA runtime.
        import torch  # noqa: F401
        lib = C.CDLL(LIB_PATH)
        P = C.POINTER
        lib.pimd_workspace_bytes.argtypes = [P(pimd_params), P(C.c_double), P(pimd_topology),
                                             P(C.c_size_t)]
        lib.pimd_create.argtypes = [P(pimd_params), P(C.c_double), P(pimd_topology), C.c_void_p,
                                    C.c_size_t, C.c_void_p, P(C.c_void_p)]
        lib.pimd_set_state.argtypes = [C.c_void_p, P(C.c_double), P(C.c_double), C.c_uint64]
        lib.pimd_step.argtypes = [C.c_void_p, C.c_int64]
        lib.pimd_get_estimators.argtypes = [C.c_void_p, P(pimd_estimators)]
        lib.pimd_get_state.argtypes = [C.c_void_p, P(C.c_double), P(C.c_double), P(C.c_uint64)]
        lib.pimd_get_barostat.argtypes = [C.c_void_p, P(C.c_double), P(C.c_double)]
        lib.pimd_boson_spring.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_double, C.c_double,
                                          P(C.c_double), C.c_void_p, C.c_void_p, C.c_void_p,
                                          C.c_void_p]
        lib.pimd_boson_spring_noalloc.argtypes = lib.pimd_boson_spring.argtypes
        lib.pimd_set_barostat.argtypes = [C.c_void_p, P(C.c_double), P(C.c_double)]
        lib.pimd_reset_averages.argtypes = [C.c_void_p]
        lib.pimd_get_positions.argtypes = [C.c_void_p, C.c_void_p]
        lib.pimd_set_forces.argtypes = [C.c_void_p, C.c_void_p, C.c_double]
        lib.pimd_destroy.argtypes = [C.c_void_p]
        lib.pimd_destroy.restype = None
        lib.pimd_profile_begin.argtypes = [C.c_void_p]
        lib.pimd_profile_end.argtypes = [C.c_void_p, P(pimd_profile)]
        lib.pimd_get_launch_info.argtypes = [C.c_void_p, P(pimd_launch_info)]
        lib.pimd_last_error.argtypes = [C.c_void_p]
        lib.pimd_last_error.restype = C.c_char_p
        lib.pimd_batch_create.argtypes = [C.c_void_p, P(C.c_void_p)]
        lib.pimd_batch_add.argtypes = [C.c_void_p, P(pimd_params), P(C.c_double), P(pimd_topology),
                                       P(C.c_int32)]
        lib.pimd_batch_remove.argtypes = [C.c_void_p, C.c_int32]
        lib.pimd_batch_set_state.argtypes = [C.c_void_p, C.c_int32, P(C.c_double), P(C.c_double),
                                             C.c_uint64]
        lib.pimd_batch_set_budget.argtypes = [C.c_void_p, C.c_int32, C.c_int64]
        lib.pimd_batch_step.argtypes = [C.c_void_p, C.c_int64]
        lib.pimd_batch_get_estimators.argtypes = [C.c_void_p, C.c_int32, P(pimd_estimators)]
        lib.pimd_batch_get_state.argtypes = [C.c_void_p, C.c_int32, P(C.c_double), P(C.c_double),
                                             P(C.c_uint64)]
        lib.pimd_batch_destroy.argtypes = [C.c_void_p]
        lib.pimd_batch_destroy.restype = None
        lib.pimd_batch_last_error.argtypes = [C.c_void_p]
        lib.pimd_batch_last_error.restype = C.c_char_p
        for n in EXPORTED:
            if n not in ("pimd_destroy", "pimd_last_error", "pimd_batch_destroy",
                         "pimd_batch_last_error"):
                getattr(lib, n).restype = C.c_int
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _estimators_dict(e) -> dict:
    out = {n: e.value[q] for q, n in enumerate(ESTIMATOR_NAMES)}
    out["step"] = e.step
    out["count"] = e.count
    out["sum"] = {n: e.sum[q] for q, n in enumerate(ESTIMATOR_NAMES)}
    out["sumsq"] = {n: e.sumsq[q] for q, n in enumerate(ESTIMATOR_NAMES)}
    out["nonfinite"], out["overflow"] = e.nonfinite, e.overflow
    out["n_rebuilds"], out["rlist"] = int(e.n_rebuilds), float(e.rlist)
    out["volume"], out["vw"], out["enthalpy"] = float(e.volume), float(e.vw), float(e.enthalpy)
    out["vwa"] = tuple(float(v) for v in e.vwa)
    return out


def _topology(lj_active, bonds, keep: list):
    if lj_active is None and bonds is None:
        return None
    t = pimd_topology()
    if lj_active is not None:
        act = np.ascontiguousarray(lj_active, dtype=np.int32)
        keep.append(act)
        t.lj_active = act.ctypes.data_as(C.POINTER(C.c_int32))
    if bonds is not None and len(bonds):
        bd = np.ascontiguousarray(bonds, dtype=np.int32).reshape(-1, 2)
        keep.append(bd)
        t.n_bonds = bd.shape[0]
        t.bonds = bd.ctypes.data_as(C.POINTER(C.c_int32))
    keep.append(t)
    return t


def params_from_spec(spec, flags: int = 0) -> pimd_params:
    """Fill pimd_params from a workload spec (``inputs.SystemSpec``)."""
    p = pimd_params()
    p.flags = int(flags)
    p.n_atoms, p.n_beads = spec.n_atoms, spec.n_beads
    p.ensemble, p.potential = int(spec.ensemble), int(spec.potential)
    p.temp, p.kB, p.hbar, p.mvv2e = spec.temp, spec.kB, spec.hbar, spec.mvv2e
    p.dt, p.tau, p.tau_scale = spec.dt, spec.tau, spec.tau_scale
    p.box = (C.c_double * 3)(*spec.box)
    p.seed = int(spec.seed) & (2**64 - 1)
    p.omega = spec.omega
    p.lj_eps, p.lj_sigma, p.lj_rc = spec.lj_eps, spec.lj_sigma, spec.lj_rc
    p.skin, p.bond_k, p.bond_r0 = spec.skin, spec.bond_k, spec.bond_r0
    p.integrator = int(getattr(spec, "integrator", PIMD_BAOAB))
    p.fixcom = int(getattr(spec, "fixcom", 0))
    p.p_ext = float(getattr(spec, "p_ext", 0.0))
    p.tau_p = float(getattr(spec, "tau_p", 1.0))
    p.bosonic = int(getattr(spec, "bosonic", 0))
    p.baro_aniso = int(getattr(spec, "baro_aniso", 0))
    return p


def boson_spring(x, kspring: float, beta_n: float, box=None, with_prob: bool = True,
                 noalloc: bool = False):
    """Bosonic exchange springs on the GPU (pimd_boson_spring) for bead
    positions x ([P][N][3], float64; a torch CUDA tensor, or host data copied
    to the device): returns V_B, EV_B (the primitive estimator's weighted
    ring energy), the spring forces [P][N][3] and the link probabilities
    [N][N] (None without with_prob).  box: periodic box lengths of the
    links' minimum image.  noalloc: pimd_boson_spring_noalloc (the library's
    static scratch, N <= 512).  Runs on torch's current stream."""
    import torch
    lib = load()
    xd = torch.as_tensor(x, dtype=torch.float64, device="cuda").contiguous()
    P, N, _ = xd.shape
    f = torch.empty_like(xd)
    prob = torch.empty((N, N), dtype=torch.float64, device="cuda") if with_prob else None
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    bx = None if box is None else (C.c_double * 3)(*[float(b) for b in box])
    stream = torch.cuda.current_stream().cuda_stream
    fn = lib.pimd_boson_spring_noalloc if noalloc else lib.pimd_boson_spring
    rc = fn(xd.data_ptr(), int(N), int(P), float(kspring), float(beta_n), bx, f.data_ptr(),
            prob.data_ptr() if prob is not None else None, out.data_ptr(), C.c_void_p(stream))
    if rc != PIMD_OK:
        msg = lib.pimd_last_error(None)
        raise PimdError(rc, msg.decode() if msg else "")
    o = out.cpu().numpy()
    return float(o[0]), float(o[1]), f, prob


class Context:
    """One ring-polymer system on the GPU (wraps a ``pimd_ctx``)."""

    def __init__(self, params: pimd_params, mass: np.ndarray, lj_active=None, bonds=None,
                 stream=None, use_torch_workspace: bool = True):
        lib = load()
        self._lib = lib
        self.params = params
        self.N, self.P = params.n_atoms, params.n_beads
        self._mass = np.ascontiguousarray(mass, dtype=np.float64)
        self._topo = None
        if lj_active is not None or bonds is not None:
            t = pimd_topology()
            if lj_active is not None:
                self._act = np.ascontiguousarray(lj_active, dtype=np.int32)
                t.lj_active = self._act.ctypes.data_as(C.POINTER(C.c_int32))
            if bonds is not None and len(bonds):
                self._bonds = np.ascontiguousarray(bonds, dtype=np.int32).reshape(-1, 2)
                t.n_bonds = self._bonds.shape[0]
                t.bonds = self._bonds.ctypes.data_as(C.POINTER(C.c_int32))
            self._topo = t
        topo = C.byref(self._topo) if self._topo is not None else None
        nbytes = C.c_size_t()
        self._check(lib.pimd_workspace_bytes(C.byref(params), _dp(self._mass), topo,
                                             C.byref(nbytes)), None)
        self.workspace_bytes = nbytes.value
        self._ws = None
        ws_ptr = None
        if use_torch_workspace:
            import torch
            # 256-byte aligned device buffer from torch's caching allocator
            self._ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device="cuda")
            base = self._ws.data_ptr()
            ws_ptr = (base + 255) & ~255
        h = C.c_void_p()
        self._check(lib.pimd_create(C.byref(params), _dp(self._mass), topo,
                                    C.c_void_p(ws_ptr) if ws_ptr else None,
                                    C.c_size_t(self.workspace_bytes + (0 if ws_ptr is None else 0)),
                                    C.c_void_p(stream) if stream else None, C.byref(h)), None)
        self._h = h

    @classmethod
    def from_spec(cls, spec, flags: int = 0, **kw) -> "Context":
        return cls(params_from_spec(spec, flags), spec.mass, lj_active=spec.lj_active,
                   bonds=spec.bonds, **kw)

    def _check(self, rc: int, h) -> None:
        if rc != PIMD_OK:
            msg = self._lib.pimd_last_error(h)
            raise PimdError(rc, msg.decode() if msg else "")

    def set_state(self, x: np.ndarray, v: np.ndarray, step: int = 0) -> None:
        x = np.ascontiguousarray(x, dtype=np.float64)
        v = np.ascontiguousarray(v, dtype=np.float64)
        assert x.shape == (self.P, self.N, 3) and v.shape == x.shape
        self._check(self._lib.pimd_set_state(self._h, _dp(x), _dp(v), int(step)), self._h)

    def step(self, n: int = 1) -> None:
        self._check(self._lib.pimd_step(self._h, int(n)), self._h)

    def estimators(self, check: bool = True) -> dict:
        e = pimd_estimators()
        rc = self._lib.pimd_get_estimators(self._h, C.byref(e))
        if check:
            self._check(rc, self._h)
        return _estimators_dict(e)

    def get_state(self):
        x = np.empty((self.P, self.N, 3))
        p = np.empty((self.P, self.N, 3))
        s = C.c_uint64()
        self._check(self._lib.pimd_get_state(self._h, _dp(x), _dp(p), C.byref(s)), self._h)
        return x, p, int(s.value)

    def barostat(self):
        """NPT, NPH: the current box lengths and barostat velocity: v_W (a
        float), or with the anisotropic barostat the three v_Wa (a tuple)."""
        box = np.empty(3)
        vw = np.zeros(3)
        self._check(self._lib.pimd_get_barostat(self._h, _dp(box), _dp(vw)), self._h)
        if self.params.baro_aniso:
            return tuple(box.tolist()), tuple(vw.tolist())
        return tuple(box.tolist()), float(vw[0])

    def set_barostat(self, box, vw) -> None:
        """NPT, NPH: the box and v_W (a float, or three with the anisotropic
        barostat) that the next set_state starts from."""
        b = np.ascontiguousarray(box, dtype=np.float64)
        v = np.ascontiguousarray(np.atleast_1d(np.asarray(vw, dtype=np.float64)))
        if v.size != (3 if self.params.baro_aniso else 1):
            raise ValueError("vw: one value, or three with the anisotropic barostat")
        self._check(self._lib.pimd_set_barostat(self._h, _dp(b), _dp(v)), self._h)

    def profile_begin(self) -> None:
        self._check(self._lib.pimd_profile_begin(self._h), self._h)

    def profile_end(self) -> dict:
        """{kernel: (launches, summed ms)} of the steps enqueued since profile_begin."""
        r = pimd_profile()
        self._check(self._lib.pimd_profile_end(self._h, C.byref(r)), self._h)
        return {n: (int(r.launches[q]), float(r.ms[q])) for q, n in enumerate(KERNEL_NAMES)}

    def launch_info(self) -> dict:
        """Launch shapes of this context (transform variant, grids, sub-groups, cells)."""
        r = pimd_launch_info()
        self._check(self._lib.pimd_get_launch_info(self._h, C.byref(r)), self._h)
        return {f: int(getattr(r, f)) for f, _ in pimd_launch_info._fields_}

    def reset_averages(self) -> None:
        self._check(self._lib.pimd_reset_averages(self._h), self._h)

    def _device_array(self, t) -> C.c_void_p:
        import torch
        assert isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
        assert t.is_contiguous() and tuple(t.shape) == (self.P, self.N, 3)
        return C.c_void_p(t.data_ptr())

    def get_positions(self, out) -> None:
        """Enqueue a copy of the positions into ``out`` (float64 CUDA tensor
        [P][N][3]); synchronize (e.g. ``torch.cuda.synchronize()``) before
        reading it."""
        self._check(self._lib.pimd_get_positions(self._h, self._device_array(out)), self._h)

    def set_forces(self, f, epot: float) -> None:
        """External potential: forces (float64 CUDA tensor [P][N][3]) on the
        current positions and their total energy sum_k U^(k)."""
        self._check(self._lib.pimd_set_forces(self._h, self._device_array(f), float(epot)), self._h)

    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.pimd_destroy(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """Many independent systems stepped together (wraps a ``pimd_batch``)."""

    def __init__(self, stream=None):
        self._lib = load()
        h = C.c_void_p()
        self._check(self._lib.pimd_batch_create(C.c_void_p(stream) if stream else None,
                                                C.byref(h)), None)
        self._h = h
        self.shapes = {}

    def _check(self, rc: int, h) -> None:
        if rc != PIMD_OK:
            msg = self._lib.pimd_batch_last_error(h)
            raise PimdError(rc, msg.decode() if msg else "")

    def add(self, spec, flags: int = 0) -> int:
        keep = []
        p = params_from_spec(spec, flags)
        mass = np.ascontiguousarray(spec.mass, dtype=np.float64)
        topo = _topology(spec.lj_active, spec.bonds, keep)
        sid = C.c_int32()
        self._check(self._lib.pimd_batch_add(self._h, C.byref(p), _dp(mass),
                                             C.byref(topo) if topo is not None else None,
                                             C.byref(sid)), self._h)
        self.shapes[sid.value] = (spec.n_beads, spec.n_atoms)
        return sid.value

    def remove(self, sid: int) -> None:
        self._check(self._lib.pimd_batch_remove(self._h, sid), self._h)
        self.shapes.pop(sid, None)

    def set_state(self, sid: int, x, v, step: int = 0) -> None:
        x = np.ascontiguousarray(x, dtype=np.float64)
        v = np.ascontiguousarray(v, dtype=np.float64)
        assert x.shape == self.shapes[sid] + (3,) and v.shape == x.shape
        self._check(self._lib.pimd_batch_set_state(self._h, sid, _dp(x), _dp(v), int(step)),
                    self._h)

    def set_budget(self, sid: int, steps: int) -> None:
        self._check(self._lib.pimd_batch_set_budget(self._h, sid, int(steps)), self._h)

    def step(self, n: int = 1) -> None:
        self._check(self._lib.pimd_batch_step(self._h, int(n)), self._h)

    def estimators(self, sid: int, check: bool = True) -> dict:
        e = pimd_estimators()
        rc = self._lib.pimd_batch_get_estimators(self._h, sid, C.byref(e))
        if check:
            self._check(rc, self._h)
        return _estimators_dict(e)

    def get_state(self, sid: int):
        P, N = self.shapes[sid]
        x = np.empty((P, N, 3))
        p = np.empty((P, N, 3))
        s = C.c_uint64()
        self._check(self._lib.pimd_batch_get_state(self._h, sid, _dp(x), _dp(p), C.byref(s)),
                    self._h)
        return x, p, int(s.value)

    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.pimd_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
