"""Seeded synthetic polyethylene melts (input generation only).

The paper simulates united-atom polyethylene: linear chains of 300 sites, 298 CH2
(type 0) with a CH3 (type 1) at each end (Section 2).  Its own initial structures
are not available, so melts are grown here from a recipe:

* cubic periodic box sized from the chain count and a mass density;
* each chain starts at a uniform point, its first bond points uniformly on the
  sphere, the second makes the tetrahedral angle with uniform azimuth, and every
  later atom takes a dihedral of 180 deg (p = 0.6), +60 deg (0.2) or -60 deg (0.2),
  bond 1.53 A, angle 109.47 deg;
* self-avoidance: a placement closer than ``d_min`` to any placed atom, other
  than the same chain's three predecessors, is rejected; up to 50 draws are made
  and the first clear one is taken; a chain stuck at a site regrows its last few
  atoms (bounded backtracking) before falling back to the draw with the largest
  clearance; chains grow in lock-step so crowding is spread over the box
  (the growth loop is plain C in ``grow.c``, seeded SplitMix64);
* Maxwell velocities at temperature T, centre-of-mass velocity removed, then
  rescaled to exactly T with 3N - 3 degrees of freedom.

Units: Angstrom, fs, g/mol, kcal/mol, K.  All randomness is seeded per melt
(SplitMix64 for growth, numpy PCG64 for velocities and jitter), so the CPU reference and the GPU library receive byte-identical
inputs.  No part of the simulation's arithmetic lives here.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import ctypes
import os
import subprocess

import numpy as np

AVOGADRO = 6.02214076e23
R_KCAL = 1.987204259e-3            # gas constant, kcal/mol/K
ACC_UNIT = 4.184e-4                # (kcal/mol/A) / (g/mol) -> A/fs^2

BOND = 1.53
ANGLE_DEG = 109.47
DIHEDRAL_STATES_DEG = (180.0, 60.0, -60.0)
DIHEDRAL_PROBS = (0.6, 0.2, 0.2)


@dataclass
class Melt:
    pos: np.ndarray        # float64 [3, N], wrapped into [0, L)
    vel: np.ndarray        # float64 [3, N], A/fs
    types: np.ndarray      # uint8 [N]
    box: np.ndarray        # float64 [3]
    n_chains: int
    chain_len: int
    T: float
    info: dict = field(default_factory=dict)

    @property
    def n_atoms(self) -> int:
        return self.pos.shape[1]


def chain_mass(chain_len: int, masses=(14.027, 15.035)) -> float:
    return (chain_len - 2) * masses[0] + 2 * masses[1]


def box_length(n_chains: int, chain_len: int, density_g_cm3: float, masses=(14.027, 15.035)) -> float:
    grams = n_chains * chain_mass(chain_len, masses) / AVOGADRO
    vol_a3 = grams / density_g_cm3 * 1e24
    return vol_a3 ** (1.0 / 3.0)


def atom_types(n_chains: int, chain_len: int) -> np.ndarray:
    t = np.zeros((n_chains, chain_len), dtype=np.uint8)
    t[:, 0] = 1
    t[:, -1] = 1
    return t.reshape(-1)


def wrap_positions(p: np.ndarray, L: np.ndarray) -> np.ndarray:
    """Wrap into [0, L) per dimension (result strictly below L)."""
    w = p - L[:, None] * np.floor(p / L[:, None])
    w = np.where(w >= L[:, None], w - L[:, None], w)
    w = np.where(w < 0.0, w + L[:, None], w)
    return w


_LIB = None
_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libgrow.so")


def build_native(force: bool = False) -> str:
    """Compile the chain grower (plain C) next to this file and return the library path."""
    src = os.path.join(_HERE, "grow.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-shared", "-fPIC",
                               src, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _lib():
    global _LIB
    if _LIB is None:
        lib = ctypes.CDLL(build_native())
        lib.pe_grow_melt.restype = ctypes.c_int
        lib.pe_grow_melt.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_uint64,
                                     ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_void_p, ctypes.c_void_p]
        _LIB = lib
    return _LIB


def _grow(n_chains: int, chain_len: int, L: float, seed: int, d_min: float, n_draws: int,
          max_depth: int = 6, max_attempts: int = 36):
    N = n_chains * chain_len
    P = np.zeros((N, 3), dtype=np.float64)
    st = np.zeros(3, dtype=np.int64)
    rc = _lib().pe_grow_melt(n_chains, chain_len, float(L), int(seed) & (2**64 - 1), float(d_min),
                             int(n_draws), int(max_depth), int(max_attempts),
                             P.ctypes.data, st.ctypes.data)
    if rc != 0:
        raise RuntimeError("pe_grow_melt failed with %d" % rc)
    return P, {"forced": int(st[0]), "backtracks": int(st[1]), "min_clearance": st[2] * 1e-6}


def maxwell_velocities(types: np.ndarray, masses, T: float, rng: np.random.Generator) -> np.ndarray:
    m = np.asarray(masses, dtype=np.float64)[types]
    N = types.size
    v = rng.normal(size=(3, N)) * np.sqrt(R_KCAL * T * ACC_UNIT / m)[None, :]
    vcom = (v * m[None, :]).sum(axis=1) / m.sum()
    v -= vcom[:, None]
    ke = 0.5 * np.sum(m[None, :] * v * v) / ACC_UNIT
    t_now = 2.0 * ke / ((3 * N - 3) * R_KCAL)
    if T > 0 and t_now > 0:
        v *= np.sqrt(T / t_now)
    return v


def make_melt(n_chains: int, chain_len: int = 300, density: float = 0.80, T: float = 500.0,
              seed_melt: int = 1000, seed_vel: int = 1001, d_min: float = 2.5,
              n_draws: int = 50, masses=(14.027, 15.035), jitter: float = 0.0,
              seed_jitter: int | None = None) -> Melt:
    """Grow a periodic polyethylene melt.  ``jitter`` (A) adds seeded Gaussian noise to
    every coordinate after growth, so bonded terms start away from their minima."""
    L = box_length(n_chains, chain_len, density, masses)
    P, stats = _grow(n_chains, chain_len, L, seed_melt, d_min, n_draws)
    Lv = np.array([L, L, L])
    pos = P.T.copy()
    if jitter > 0:
        jr = np.random.default_rng(seed_melt + 7919 if seed_jitter is None else seed_jitter)
        pos = pos + jr.normal(scale=jitter, size=pos.shape)
    pos = np.ascontiguousarray(wrap_positions(pos, Lv))
    types = atom_types(n_chains, chain_len)
    vel = np.ascontiguousarray(maxwell_velocities(types, masses, T, np.random.default_rng(seed_vel)))
    return Melt(pos=pos, vel=vel, types=types, box=Lv, n_chains=n_chains,
                chain_len=chain_len, T=T, info={"density": density, "seed_melt": seed_melt,
                                                 "seed_vel": seed_vel, **stats})


def unwrap_chains(pos: np.ndarray, box: np.ndarray, chain_len: int) -> np.ndarray:
    """Undo the wrap along each chain (consecutive atoms closer than half a box)."""
    N = pos.shape[1]
    p = pos.T.reshape(-1, chain_len, 3)
    d = np.diff(p, axis=1)
    d -= box * np.round(d / box)
    out = np.concatenate([p[:, :1], p[:, :1] + np.cumsum(d, axis=1)], axis=1)
    return out.reshape(N, 3).T


def make_tiled_melt(n_chains: int, tiles: int, chain_len: int = 300, density: float = 0.80,
                    T: float = 500.0, seed_melt: int = 1000, seed_vel: int = 1001, d_min: float = 2.5,
                    n_draws: int = 50, masses=(14.027, 15.035)) -> Melt:
    """A large melt as tiles^3 copies of one grown in a box tiles times smaller per edge.

    The small melt's chains are unwrapped and copied to every cell of a tiles x tiles x tiles
    lattice of small boxes, then wrapped into the large box.  Every atom then sees exactly the
    neighbourhood it had in the small periodic box, so bonds, clearances and density carry
    over; the copies differ through their velocities, drawn for the whole system.  Chains are
    numbered copy by copy.  (Growing 3-30 million atoms site by site takes minutes; this
    takes seconds.)"""
    if tiles < 1 or n_chains % (tiles ** 3):
        raise ValueError("n_chains must be a multiple of tiles^3")
    small = make_melt(n_chains // tiles ** 3, chain_len, density, T, seed_melt, seed_vel, d_min, n_draws, masses)
    Ls = small.box
    base = unwrap_chains(small.pos, Ls, chain_len)
    shifts = np.array([(a, b, c) for a in range(tiles) for b in range(tiles) for c in range(tiles)], dtype=np.float64)
    pos = (base[:, None, :] + (shifts.T * Ls[:, None])[:, :, None]).reshape(3, -1)
    L = Ls * tiles
    pos = np.ascontiguousarray(wrap_positions(pos, L))
    types = atom_types(n_chains, chain_len)
    vel = np.ascontiguousarray(maxwell_velocities(types, masses, T, np.random.default_rng(seed_vel)))
    info = {k: v for k, v in small.info.items()}
    info.update({"density": density, "tiles": tiles, "tile_box": float(Ls[0])})
    return Melt(pos=pos, vel=vel, types=types, box=L, n_chains=n_chains, chain_len=chain_len, T=T, info=info)
