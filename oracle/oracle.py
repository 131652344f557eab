"""ctypes binding of ``oracle_md.c`` (test infrastructure only; see ``oracle_md.h``).

Arrays are numpy: positions/velocities/forces float64 [3, N] (structure of arrays),
types uint8 [N].  Every function copies what it modifies, so callers' arrays are
never changed behind their back.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle_md.c")
_SO = os.path.join(_HERE, "liboracle.so")
_LIB = None

D = ctypes.c_double
I32 = ctypes.c_int32
I64 = ctypes.c_int64
P = ctypes.c_void_p


class OraFF(ctypes.Structure):
    _fields_ = [("mass", D * 2), ("sigma", D * 2), ("epsilon", D * 2), ("kb", D), ("b0", D),
                ("ka", D), ("theta0_deg", D), ("kphi", D), ("phis_deg", D), ("n_dih", I32),
                ("rc", D), ("excl_depth", I32)]


class OraEnergy(ctypes.Structure):
    _fields_ = [("e_lj", D), ("e_lj_shifted", D), ("e_bond", D), ("e_angle", D), ("e_dih", D),
                ("virial_lj", D), ("virial_bonded", D)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class OraInteg(ctypes.Structure):
    _fields_ = [("dt", D), ("tau", D), ("T0", D), ("remove_com", I32)]


class OraNH(ctypes.Structure):
    _fields_ = [("xi", D), ("eta", D), ("e_thermostat", D)]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no FP contraction, OpenMP)."""
    hdr = os.path.join(_HERE, "oracle_md.h")
    newest = max(os.path.getmtime(_SRC), os.path.getmtime(hdr))
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < newest:
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fopenmp",
                               "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _LIB
    if _LIB is None:
        L = ctypes.CDLL(build())
        sig = {
            "ora_set_threads": (ctypes.c_int, [ctypes.c_int]),
            "ora_wrap": (ctypes.c_int, [I64, P, P, P, P]),
            "ora_cell_index": (ctypes.c_int, [I64, P, P, P, P, P, P]),
            "ora_bin": (ctypes.c_int, [I64, P, I64, P, P, P]),
            "ora_lj_brute": (ctypes.c_int, [P, I64, I32, P, P, P, P, P, P, P, P, P]),
            "ora_lj_cells": (ctypes.c_int, [P, I64, I32, P, P, P, P, P, P, I32, P, I64, P, P, P, P]),
            "ora_bonded": (ctypes.c_int, [P, I64, I32, P, P, P, P, P, P, P, P]),
            "ora_forces": (ctypes.c_int, [P, I64, I32, P, P, P, P, P, P, I32, P, P, P, P]),
            "ora_sum": (D, [I64, P]),
            "ora_chain_terms": (ctypes.c_int, [I32, I32, P, I32]),
            "ora_kinetic": (ctypes.c_int, [P, I64, P, P, P, P, P, P]),
            "ora_bond_term": (D, [P, P, P, P]),
            "ora_angle_term": (D, [P, P, P, P, P, P]),
            "ora_dihedral_term": (D, [P, P, P, P, P, P, P]),
            "ora_run": (ctypes.c_int, [P, P, I64, I32, P, P, P, P, P, P, P, P, P, P, P, P, I32, I32,
                                       P, P, P]),
            "ora_run_leapfrog": (ctypes.c_int, [P, P, P, I64, I32, P, P, P, P, P, P, P, P, P, P, P, P, I32,
                                                I32, P, P, P]),
            "ora_com_velocity": (ctypes.c_int, [P, I64, P, P, P, P, P]),
            "ora_pair_histogram": (ctypes.c_int, [I64, I32, I32, P, P, P, P, P, D, I32, P]),
            "ora_dihedral_stats": (ctypes.c_int, [I64, I32, P, P, P, P, I32, P, P]),
            "ora_chain_shape": (ctypes.c_int, [P, I64, I32, P, P, P, P, P, P]),
            "ora_ree_acf": (ctypes.c_int, [I64, I32, P, P, P, P, P, P, P, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def _p(a):
    return a.ctypes.data if a is not None else None


def _check(rc, what):
    if rc != 0:
        raise RuntimeError("%s failed with status %d" % (what, rc))


def make_ff(ff: dict) -> OraFF:
    s = OraFF()
    s.mass[:] = ff["mass"]
    s.sigma[:] = ff["sigma"]
    s.epsilon[:] = ff["epsilon"]
    for k in ("kb", "b0", "ka", "theta0_deg", "kphi", "phis_deg", "rc"):
        setattr(s, k, float(ff[k]))
    s.n_dih = int(ff["n_dih"])
    s.excl_depth = int(ff["excl_depth"])
    return s


def _soa(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    assert a.ndim == 2 and a.shape[0] == 3
    return a


def _box(box):
    return np.ascontiguousarray(np.broadcast_to(np.asarray(box, dtype=np.float64), (3,)))


def set_threads(n: int) -> int:
    return lib().ora_set_threads(int(n))


def grid_dims(box, rc: float, R: int = 1) -> np.ndarray:
    """Cells per dimension for a stencil of radius R: M = floor(L R / rc), edge L/M >= rc/R."""
    L = _box(box)
    return np.floor(L * R / rc).astype(np.int32)


def wrap(pos, box):
    p = _soa(pos).copy()
    L = _box(box)
    _check(lib().ora_wrap(p.shape[1], _p(p[0]), _p(p[1]), _p(p[2]), _p(L)), "ora_wrap")
    return p


def cell_index(pos, box, M):
    p = _soa(pos)
    L = _box(box)
    Mv = np.ascontiguousarray(M, dtype=np.int32)
    cell = np.empty(p.shape[1], dtype=np.int32)
    _check(lib().ora_cell_index(p.shape[1], _p(p[0]), _p(p[1]), _p(p[2]), _p(L), _p(Mv), _p(cell)),
           "ora_cell_index")
    return cell


def bin_atoms(cell, n_cells):
    cell = np.ascontiguousarray(cell, dtype=np.int32)
    cnt = np.empty(n_cells, dtype=np.int32)
    start = np.empty(n_cells + 1, dtype=np.int32)
    atoms = np.empty(cell.size, dtype=np.int32)
    _check(lib().ora_bin(cell.size, _p(cell), n_cells, _p(cnt), _p(start), _p(atoms)), "ora_bin")
    return cnt, start, atoms


def lj_brute(ff, pos, types, box, chain_len):
    p = _soa(pos)
    t = np.ascontiguousarray(types, dtype=np.uint8)
    L = _box(box)
    f = np.zeros_like(p)
    e = OraEnergy()
    s = make_ff(ff)
    _check(lib().ora_lj_brute(ctypes.byref(s), p.shape[1], chain_len, _p(p[0]), _p(p[1]), _p(p[2]),
                              _p(t), _p(L), _p(f[0]), _p(f[1]), _p(f[2]), ctypes.byref(e)),
           "ora_lj_brute")
    return f, e.as_dict()


def lj_cells(ff, pos, types, box, chain_len, M=None, R=1, subset=None):
    p = _soa(pos)
    t = np.ascontiguousarray(types, dtype=np.uint8)
    L = _box(box)
    Mv = np.ascontiguousarray(grid_dims(L, ff["rc"], R) if M is None else M, dtype=np.int32)
    f = np.zeros_like(p)
    e = OraEnergy()
    s = make_ff(ff)
    sub = None if subset is None else np.ascontiguousarray(subset, dtype=np.int64)
    _check(lib().ora_lj_cells(ctypes.byref(s), p.shape[1], chain_len, _p(p[0]), _p(p[1]), _p(p[2]),
                              _p(t), _p(L), _p(Mv), int(R), _p(sub), 0 if sub is None else sub.size,
                              _p(f[0]), _p(f[1]), _p(f[2]), ctypes.byref(e)), "ora_lj_cells")
    if sub is not None:
        return f[:, sub], None
    return f, e.as_dict()


def bonded(ff, pos, box, chain_len):
    p = _soa(pos)
    L = _box(box)
    f = np.zeros_like(p)
    e = OraEnergy()
    s = make_ff(ff)
    _check(lib().ora_bonded(ctypes.byref(s), p.shape[1], chain_len, _p(p[0]), _p(p[1]), _p(p[2]),
                            _p(L), _p(f[0]), _p(f[1]), _p(f[2]), ctypes.byref(e)), "ora_bonded")
    d = e.as_dict()
    return f, {k: d[k] for k in ("e_bond", "e_angle", "e_dih", "virial_bonded")}


def forces(ff, pos, types, box, chain_len, M=None, R=1):
    p = _soa(pos)
    t = np.ascontiguousarray(types, dtype=np.uint8)
    L = _box(box)
    Mv = np.ascontiguousarray(grid_dims(L, ff["rc"], R) if M is None else M, dtype=np.int32)
    f = np.zeros_like(p)
    e = OraEnergy()
    s = make_ff(ff)
    _check(lib().ora_forces(ctypes.byref(s), p.shape[1], chain_len, _p(p[0]), _p(p[1]), _p(p[2]),
                            _p(t), _p(L), _p(Mv), int(R), _p(f[0]), _p(f[1]), _p(f[2]),
                            ctypes.byref(e)), "ora_forces")
    return f, e.as_dict()


def chain_terms(chain_len: int, k: int) -> np.ndarray:
    """0-based site tuples of the k-site terms (2 bond, 3 angle, 4 dihedral) of one chain."""
    out = np.zeros((max(chain_len, 1), k), dtype=np.int32)
    m = lib().ora_chain_terms(int(chain_len), int(k), _p(out), out.shape[0])
    if m < 0:
        raise RuntimeError("ora_chain_terms failed")
    return out[:m].copy()


def compensated_sum(v):
    v = np.ascontiguousarray(v, dtype=np.float64)
    return lib().ora_sum(v.size, _p(v))


def kinetic(ff, vel, types):
    v = _soa(vel)
    t = np.ascontiguousarray(types, dtype=np.uint8)
    ke, T = D(), D()
    s = make_ff(ff)
    _check(lib().ora_kinetic(ctypes.byref(s), v.shape[1], _p(v[0]), _p(v[1]), _p(v[2]), _p(t),
                             ctypes.byref(ke), ctypes.byref(T)), "ora_kinetic")
    return ke.value, T.value


def bond_term(ff, xi, xj):
    f = np.zeros(6)
    s = make_ff(ff)
    a = [np.ascontiguousarray(v, dtype=float) for v in (xi, xj)]
    e = lib().ora_bond_term(ctypes.byref(s), _p(a[0]), _p(a[1]), _p(f))
    return e, f.reshape(2, 3)


def angle_term(ff, xi, xj, xk):
    f = np.zeros(9)
    th = D()
    s = make_ff(ff)
    a = [np.ascontiguousarray(v, dtype=float) for v in (xi, xj, xk)]
    e = lib().ora_angle_term(ctypes.byref(s), _p(a[0]), _p(a[1]), _p(a[2]), _p(f), ctypes.byref(th))
    return e, f.reshape(3, 3), th.value


def dihedral_term(ff, xi, xj, xk, xl):
    f = np.zeros(12)
    ph = D()
    s = make_ff(ff)
    a = [np.ascontiguousarray(v, dtype=float) for v in (xi, xj, xk, xl)]
    e = lib().ora_dihedral_term(ctypes.byref(s), _p(a[0]), _p(a[1]), _p(a[2]), _p(a[3]), _p(f),
                                ctypes.byref(ph))
    return e, f.reshape(4, 3), ph.value


def com_velocity(ff, vel, types):
    """Centre-of-mass velocity of the atoms, sum m v / sum m."""
    v = _soa(vel)
    t = np.ascontiguousarray(types, dtype=np.uint8)
    u = np.zeros(3)
    s = make_ff(ff)
    _check(lib().ora_com_velocity(ctypes.byref(s), v.shape[1], _p(v[0]), _p(v[1]), _p(v[2]), _p(t), _p(u)),
           "ora_com_velocity")
    return u


def run_leapfrog(ff, pos, vel, frc, types, box, chain_len, n_steps, dt=1.0, tau=100.0, T0=0.0, M=None, R=1,
                 remove_com=False, nh=(0.0, 0.0)):
    """Leap-frog + Nose-Hoover on copies of (pos, vel, frc): vel holds v(t - dt/2) and frc
    the force at pos.  nh = (xi, eta) on entry.  Returns (pos, vel, frc, energies) with the
    energies dict carrying xi, eta and e_thermostat after the last step."""
    p = _soa(pos).copy()
    v = _soa(vel).copy()
    f = _soa(frc).copy()
    t = np.ascontiguousarray(types, dtype=np.uint8)
    L = _box(box)
    Mv = np.ascontiguousarray(grid_dims(L, ff["rc"], R) if M is None else M, dtype=np.int32)
    e = OraEnergy()
    ke, T = D(), D()
    s = make_ff(ff)
    integ = OraInteg(dt=dt, tau=tau, T0=T0, remove_com=1 if remove_com else 0)
    st = OraNH(xi=nh[0], eta=nh[1], e_thermostat=0.0)
    _check(lib().ora_run_leapfrog(ctypes.byref(s), ctypes.byref(integ), ctypes.byref(st), p.shape[1], chain_len,
                                  _p(p[0]), _p(p[1]), _p(p[2]), _p(v[0]), _p(v[1]), _p(v[2]),
                                  _p(f[0]), _p(f[1]), _p(f[2]), _p(t), _p(L), _p(Mv), int(R), int(n_steps),
                                  ctypes.byref(e), ctypes.byref(ke), ctypes.byref(T)), "ora_run_leapfrog")
    return p, v, f, {**e.as_dict(), "e_kin": ke.value, "temperature": T.value, "xi": st.xi, "eta": st.eta,
                     "e_thermostat": st.e_thermostat}


def pair_histogram(pos, box, chain_len, excl_depth, rmax, n_bins, cells=True):
    """Unordered non-excluded pairs per distance bin over [0, rmax) (grid search, or brute
    force with cells=False).  Positions must be wrapped for the grid search."""
    p = _soa(pos)
    L = _box(box)
    out = np.zeros(int(n_bins), dtype=np.uint64)
    M = None
    if cells:
        M = np.ascontiguousarray(np.floor(L / rmax).astype(np.int32))
    _check(lib().ora_pair_histogram(p.shape[1], int(chain_len), int(excl_depth), _p(p[0]), _p(p[1]), _p(p[2]),
                                    _p(L), _p(M) if M is not None else None, float(rmax), int(n_bins), _p(out)),
           "ora_pair_histogram")
    return out


def dihedral_stats(pos, box, chain_len, n_bins):
    """(histogram of the IUPAC dihedral angle over (-pi, pi], [trans, gauche+, gauche-])."""
    p = _soa(pos)
    L = _box(box)
    hist = np.zeros(max(int(n_bins), 1), dtype=np.uint64)
    cls = np.zeros(3, dtype=np.uint64)
    _check(lib().ora_dihedral_stats(p.shape[1], int(chain_len), _p(p[0]), _p(p[1]), _p(p[2]), _p(L), int(n_bins),
                                    _p(hist), _p(cls)), "ora_dihedral_stats")
    return hist[:int(n_bins)], cls


def chain_shape(ff, pos, types, box, chain_len):
    """[n_chains, 4]: mass-weighted Rg^2 and the end-to-end vector of each chain."""
    p = _soa(pos)
    t = np.ascontiguousarray(types, dtype=np.uint8)
    L = _box(box)
    out = np.zeros((p.shape[1] // int(chain_len), 4))
    s = make_ff(ff)
    _check(lib().ora_chain_shape(ctypes.byref(s), p.shape[1], int(chain_len), _p(p[0]), _p(p[1]), _p(p[2]), _p(t),
                                 _p(L), _p(out)), "ora_chain_shape")
    return out


def ree_acf(pos0, pos, box, chain_len):
    """End-to-end vector autocorrelation sum_c R_c(t).R_c(0) / sum_c |R_c(0)|^2 (Fig. 8) between
    the positions pos0 (reference time) and pos."""
    a, b = _soa(pos0), _soa(pos)
    assert a.shape == b.shape
    L = _box(box)
    out = D()
    _check(lib().ora_ree_acf(a.shape[1], chain_len, _p(a[0]), _p(a[1]), _p(a[2]), _p(b[0]), _p(b[1]), _p(b[2]),
                             _p(L), ctypes.byref(out)), "ora_ree_acf")
    return out.value


def run(ff, pos, vel, frc, types, box, chain_len, n_steps, dt=1.0, tau=100.0, T0=0.0, M=None, R=1,
        remove_com=False):
    """Advance copies of (pos, vel, frc) by n_steps; frc must be the force at pos."""
    p = _soa(pos).copy()
    v = _soa(vel).copy()
    f = _soa(frc).copy()
    t = np.ascontiguousarray(types, dtype=np.uint8)
    L = _box(box)
    Mv = np.ascontiguousarray(grid_dims(L, ff["rc"], R) if M is None else M, dtype=np.int32)
    e = OraEnergy()
    ke, T = D(), D()
    s = make_ff(ff)
    integ = OraInteg(dt=dt, tau=tau, T0=T0, remove_com=1 if remove_com else 0)
    _check(lib().ora_run(ctypes.byref(s), ctypes.byref(integ), p.shape[1], chain_len,
                         _p(p[0]), _p(p[1]), _p(p[2]), _p(v[0]), _p(v[1]), _p(v[2]),
                         _p(f[0]), _p(f[1]), _p(f[2]), _p(t), _p(L), _p(Mv), int(R), int(n_steps),
                         ctypes.byref(e), ctypes.byref(ke), ctypes.byref(T)), "ora_run")
    return p, v, f, {**e.as_dict(), "e_kin": ke.value, "temperature": T.value}


__all__ = ["build", "lib", "make_ff", "ree_acf", "set_threads", "grid_dims", "wrap", "cell_index", "bin_atoms",
           "lj_brute", "lj_cells", "bonded", "forces", "chain_terms", "compensated_sum", "kinetic", "bond_term",
           "angle_term", "dihedral_term", "run", "run_leapfrog", "com_velocity", "pair_histogram", "dihedral_stats",
           "chain_shape"]
