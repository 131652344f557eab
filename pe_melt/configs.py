"""Workload presets: synthetic polyethylene melts of the sizes the benchmarks use.

Every preset uses 300-site chains (Section 2) and the Table I force field.  The
paper's own test systems (Table III) and its crystallisation structures are not
available, so seeded melts grown by :mod:`pe_melt.generator` stand in for them.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    n_chains: tuple            # chains per box
    density: float             # g/cm^3
    T_init: tuple              # K, per box (Maxwell draw)
    T0: tuple                  # K, per box thermostat target; <= 0 means NVE
    steps: int
    seeds: tuple               # (melt seed, velocity seed) per box
    precision: str             # "fp64" or "mixed"
    chain_len: int = 300
    dt_fs: float = 1.0
    tau_fs: float = 100.0
    tiles: int = 1             # > 1: each box is tiles^3 copies of a melt grown tiles x smaller

    @property
    def n_boxes(self) -> int:
        return len(self.n_chains)

    @property
    def n_atoms(self) -> int:
        return self.chain_len * int(sum(self.n_chains))


def _batched_ensemble(n_boxes: int = 64, lo: int = 20, hi: int = 400, seed: int = 4999) -> Workload:
    rng = np.random.default_rng(seed)
    counts = tuple(int(c) for c in rng.integers(lo, hi + 1, size=n_boxes))
    temps = tuple(250.0 + 200.0 * b / (n_boxes - 1) for b in range(n_boxes))
    seeds = tuple((4000 + 2 * b, 4001 + 2 * b) for b in range(n_boxes))
    return Workload("ensemble64_mixed", counts, 0.80, temps, temps, 2000, seeds, "mixed")


WORKLOADS = {
    # 10 chains, 3,000 atoms, plain FP64, NVE at 500 K, 100 steps
    "melt3k_fp64": Workload("melt3k_fp64", (10,), 0.80, (500.0,), (0.0,), 100, ((1000, 1001),), "fp64"),
    # 1,000 chains, 300,000 atoms, mixed precision, Berendsen quench 500 -> 300 K
    "melt300k_mixed": Workload("melt300k_mixed", (1000,), 0.80, (500.0,), (300.0,), 10000,
                               ((2000, 2001),), "mixed"),
    # 10,000 chains, 3,000,000 atoms, 0.85 g/cm^3, 300 K NVT
    "melt3M_mixed": Workload("melt3M_mixed", (10000,), 0.85, (300.0,), (300.0,), 5000,
                             ((3000, 3001),), "mixed", tiles=2),
    # 64 independent boxes of 20..400 chains at 250..450 K
    "ensemble64_mixed": _batched_ensemble(),
    # 100,000 chains, 30,000,000 atoms, 0.85 g/cm^3, 300 K NVT
    "melt30M_mixed": Workload("melt30M_mixed", (100000,), 0.85, (300.0,), (300.0,), 1000,
                              ((5000, 5001),), "mixed", tiles=5),
}


def build_melts(wl: Workload, threads: int = 16) -> list:
    """The seeded melt of every box of a workload.  Boxes are grown on a thread pool (the
    C grower runs without the interpreter lock), so a 64-box ensemble takes seconds."""
    from concurrent.futures import ThreadPoolExecutor

    from .generator import make_melt, make_tiled_melt

    def one(b: int):
        sm, sv = wl.seeds[b]
        if wl.tiles > 1:
            return make_tiled_melt(wl.n_chains[b], wl.tiles, wl.chain_len, wl.density, wl.T_init[b], sm, sv)
        return make_melt(wl.n_chains[b], wl.chain_len, wl.density, wl.T_init[b], sm, sv)

    with ThreadPoolExecutor(max_workers=max(1, min(threads, wl.n_boxes))) as ex:
        return list(ex.map(one, range(wl.n_boxes)))
