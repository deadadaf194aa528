"""Host-side checks that need no GPU: libpimd.so loads and exports every entry
point that include/pimd.h declares, the binding's structs match the header's
field order, and the seeded workload generators produce what they promise."""
import ctypes as C
import math
import os
import re
from dataclasses import replace as dataclasses_replace

import numpy as np
import pytest

from paper_2602_13553_amd import inputs, pimd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pimd.h")


def header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pimd_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    declared = header_functions()
    assert set(declared) == set(pimd.EXPORTED)
    lib = C.CDLL(pimd.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name


def test_binding_structs_follow_header():
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)

    def fields(struct):
        body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (struct, struct), src, re.S).group(1)
        names = []
        for decl in body.split(";"):
            decl = re.sub(r"\[.*?\]", "", decl).replace("*", " ")
            toks = [t for t in decl.replace(",", " , ").split() if t != "const"]
            if not toks:
                continue
            # first token is the type, then comma-separated names
            names += [t for t in toks[1:] if t != ","]
        return names

    assert fields("pimd_params") == [f[0] for f in pimd.pimd_params._fields_]
    assert fields("pimd_topology") == [f[0] for f in pimd.pimd_topology._fields_]
    assert fields("pimd_estimators") == [f[0] for f in pimd.pimd_estimators._fields_]
    assert fields("pimd_profile") == [f[0] for f in pimd.pimd_profile._fields_]
    nest = int(re.search(r"#define PIMD_NEST (\d+)", src).group(1))
    assert pimd.NEST == nest == len(pimd.ESTIMATOR_NAMES)
    assert fields("pimd_launch_info") == [f[0] for f in pimd.pimd_launch_info._fields_]


def test_create_rejects_bad_parameters_without_gpu():
    """Validation runs before any device call."""
    lib = pimd.load()
    spec = inputs.harmonic_tiny()
    p = pimd.params_from_spec(spec)
    n = C.c_size_t()
    mass = np.ascontiguousarray(spec.mass)
    assert lib.pimd_workspace_bytes(C.byref(p), pimd._dp(mass), None, C.byref(n)) == 0
    assert n.value > 0
    bad = pimd.params_from_spec(spec)
    bad.n_beads = 129
    assert lib.pimd_workspace_bytes(C.byref(bad), pimd._dp(mass), None, C.byref(n)) == -6
    bad = pimd.params_from_spec(spec)
    bad.dt = -1.0
    assert lib.pimd_workspace_bytes(C.byref(bad), pimd._dp(mass), None, C.byref(n)) == -1
    assert b"dt" in lib.pimd_last_error(None)
    lj = pimd.params_from_spec(inputs.lj_liquid(n_atoms=32, n_beads=4))
    lj.box = (C.c_double * 3)(0.0, 1.0, 1.0)
    assert lib.pimd_workspace_bytes(C.byref(lj), pimd._dp(np.ones(32)), None, C.byref(n)) == -6
    h = C.c_void_p()
    assert lib.pimd_create(C.byref(bad), pimd._dp(mass), None, None, 0, None, C.byref(h)) == -1


def test_external_potential_is_accepted_without_gpu():
    """PIMD_POT_EXTERNAL (forces from the caller) needs no box or pair
    parameters; the next code is rejected."""
    lib = pimd.load()
    spec = inputs.harmonic_tiny()
    mass = np.ascontiguousarray(spec.mass)
    n = C.c_size_t()
    p = pimd.params_from_spec(spec)
    p.potential = pimd.PIMD_POT_EXTERNAL
    assert lib.pimd_workspace_bytes(C.byref(p), pimd._dp(mass), None, C.byref(n)) == 0
    n_ext = n.value
    p.potential = pimd.PIMD_POT_HARMONIC
    assert lib.pimd_workspace_bytes(C.byref(p), pimd._dp(mass), None, C.byref(n)) == 0
    assert n_ext > n.value            # room for the caller's forces
    p.potential = pimd.PIMD_POT_EXTERNAL + 1
    assert lib.pimd_workspace_bytes(C.byref(p), pimd._dp(mass), None, C.byref(n)) == -1
    assert "#define PIMD_POT_EXTERNAL %d" % pimd.PIMD_POT_EXTERNAL in open(HEADER).read()


def test_flags_are_validated_without_gpu():
    """Launch-shape flags: unknown bits and sub-group counts beyond one block fail."""
    lib = pimd.load()
    spec = inputs.lj_liquid(n_atoms=256, n_beads=32)
    mass = np.ascontiguousarray(spec.mass)
    n = C.c_size_t()
    for flags, rc in ((pimd.PIMD_FLAG_VALU_TRANSFORMS, 0), (pimd.PIMD_FLAG_MFMA_TRANSFORMS, 0),
                      (pimd.PIMD_PAIR_SUBGROUPS(8), 0), (pimd.PIMD_PAIR_SUBGROUPS(16), -1),
                      (1 << 20, -1), (6 << pimd.PIMD_PAIR_SUBGROUPS_SHIFT, -1)):
        p = pimd.params_from_spec(spec, flags)
        assert lib.pimd_workspace_bytes(C.byref(p), pimd._dp(mass), None, C.byref(n)) == rc, flags
    # the header's macro and the binding agree on the encoding
    src = open(HEADER).read()
    assert "#define PIMD_PAIR_SUBGROUPS_SHIFT %d" % pimd.PIMD_PAIR_SUBGROUPS_SHIFT in src
    assert "#define PIMD_FLAG_MFMA_TRANSFORMS %d" % pimd.PIMD_FLAG_MFMA_TRANSFORMS in src


def test_workload_generators():
    h = inputs.harmonic_tiny()
    assert h.x0.shape == (4, 64, 3) and h.n_beads == 4 and h.temp == 0.25
    lj = inputs.lj_liquid()
    L = lj.box[0]
    assert lj.n_atoms == 4000 and abs(4000 / L ** 3 - 0.8) < 1e-12
    d = np.linalg.norm(lj.x0[0, 0] - lj.x0[0, 1:], axis=1).min()
    assert abs(d - L / 10 / math.sqrt(2)) < 0.1
    w = inputs.water()
    assert w.n_atoms == 32766 and w.extra["n_mol"] == 10922
    assert abs(w.box[0] - 68.875) < 1e-3
    x = w.x0.mean(axis=0)
    r = np.linalg.norm(x[w.bonds[:, 0]] - x[w.bonds[:, 1]], axis=1)
    assert np.allclose(r, 0.96, atol=0.05)
    assert w.lj_active.sum() == 10922
    assert abs(inputs.REAL_HBAR - 15.1787283) < 1e-6 and abs(inputs.REAL_MVV2E - 2390.0573) < 1e-3
    b = inputs.batch_systems(n_systems=64)
    ns = np.array([s.n_atoms for s in b])
    assert ns.min() >= 64 and ns.max() <= 4096
    assert set(s.n_beads for s in b) <= {8, 16, 32, 64}
    tr = inputs.serving_trace(n_jobs=200)
    gaps = np.diff([j.arrival for j in tr])
    assert abs(gaps.mean() - 1 / 20) < 0.3 / 20
    assert all(j.n_atoms % 3 == 0 for j in tr if j.kind == "water")


def test_barostat_validation_without_gpu():
    """The barostat needs a pair potential, no fixcom, tau_p > 0 and a finite
    p_ext, takes either splitting, and neither the matrix-core nor the
    cluster flags; baro_aniso is 0 or 1, and 1 only under a barostat."""
    lib = pimd.load()
    spec = inputs.lj_liquid(n_atoms=32, n_beads=4)
    mass = np.ascontiguousarray(spec.mass)
    n = C.c_size_t()

    def rc(**kw):
        p = pimd.params_from_spec(spec)
        p.ensemble, p.integrator, p.p_ext, p.tau_p = pimd.PIMD_NPT, pimd.PIMD_OBABO, 1.0, 0.5
        for k, v in kw.items():
            setattr(p, k, v)
        return lib.pimd_workspace_bytes(C.byref(p), pimd._dp(mass), None, C.byref(n))

    assert rc() == 0
    assert rc(ensemble=pimd.PIMD_NPH) == 0
    assert rc(integrator=pimd.PIMD_BAOAB) == 0
    assert rc(fixcom=1) == -6
    assert rc(tau_p=0.0) == -1
    assert rc(p_ext=float("nan")) == -1
    assert rc(flags=pimd.PIMD_FLAG_MFMA_TRANSFORMS) == -6
    assert rc(ensemble=4) == -1
    # the anisotropic barostat: 0 or 1, and only with a barostat; its
    # workspace adds the force pass's per-block diagonal virials
    assert rc() == 0
    iso = n.value
    assert rc(baro_aniso=1) == 0 and n.value > iso
    assert rc(baro_aniso=1, ensemble=pimd.PIMD_NPH, integrator=pimd.PIMD_BAOAB) == 0
    assert rc(baro_aniso=2) == -1
    assert rc(baro_aniso=1, ensemble=pimd.PIMD_NVT) == -1
    assert rc(baro_aniso=1, ensemble=pimd.PIMD_NVE) == -1
    h = pimd.params_from_spec(inputs.harmonic_tiny())
    h.ensemble, h.integrator, h.tau_p = pimd.PIMD_NPT, pimd.PIMD_OBABO, 0.5
    hm = np.ascontiguousarray(inputs.harmonic_tiny().mass)
    assert lib.pimd_workspace_bytes(C.byref(h), pimd._dp(hm), None, C.byref(n)) == -6


def test_bosonic_validation_without_gpu():
    """The bosonic fix's limits are checked before any device call: NVT or
    NVE, no water, no fixcom, no barostat, at most 1024 bosons; the trap, LJ,
    no potential and the caller's forces are accepted, and the workspace holds
    the spring forces and the exchange scratch."""
    lib = pimd.load()
    n = C.c_size_t()
    spec = inputs.trapped_bosons(n_atoms=16, n_beads=8)
    mass = np.ascontiguousarray(spec.mass)
    p = pimd.params_from_spec(spec)
    assert p.bosonic == 1
    assert lib.pimd_workspace_bytes(C.byref(p), pimd._dp(mass), None, C.byref(n)) == 0
    q = pimd.params_from_spec(dataclasses_replace(spec, bosonic=0))
    n0 = C.c_size_t()
    assert lib.pimd_workspace_bytes(C.byref(q), pimd._dp(mass), None, C.byref(n0)) == 0
    assert n.value >= n0.value + 16 * 8 * 3 * 8 + 8 * (16 * 17)
    for field, value, code in (("ensemble", pimd.PIMD_NPT, -6), ("potential", pimd.PIMD_POT_WATER, -6),
                               ("fixcom", 1, -6), ("bosonic", 2, -1)):
        bad = pimd.params_from_spec(spec)
        setattr(bad, field, value)
        assert lib.pimd_workspace_bytes(C.byref(bad), pimd._dp(mass), None, C.byref(n)) == code, field
    big = inputs.trapped_bosons(n_atoms=1025, n_beads=2)
    bp = pimd.params_from_spec(big)
    assert lib.pimd_workspace_bytes(C.byref(bp), pimd._dp(np.ascontiguousarray(big.mass)), None,
                                    C.byref(n)) == -6
    lj = inputs.lj_bosons(n_atoms=108, n_beads=4)
    lp = pimd.params_from_spec(lj)
    assert lib.pimd_workspace_bytes(C.byref(lp), pimd._dp(np.ascontiguousarray(lj.mass)), None,
                                    C.byref(n)) == 0
    for pot in (pimd.PIMD_POT_NONE, pimd.PIMD_POT_EXTERNAL):
        ok = pimd.params_from_spec(spec)
        ok.potential = pot
        assert lib.pimd_workspace_bytes(C.byref(ok), pimd._dp(mass), None, C.byref(n)) == 0, pot
