"""Seeded synthetic inputs (polyethylene melts, force-field parameters, workload presets).

Shared as input data by the CPU reference (``oracle/``) and the GPU library; it holds
none of the simulation's arithmetic.
"""

from .configs import WORKLOADS, Workload, build_melts
from .forcefield import polyethylene_forcefield, table_i_in_kcal_angstrom
from .generator import Melt, box_length, make_melt, make_tiled_melt, unwrap_chains, wrap_positions

__all__ = ["WORKLOADS", "Workload", "build_melts", "Melt", "box_length", "make_melt", "make_tiled_melt", "unwrap_chains",
           "wrap_positions", "polyethylene_forcefield", "table_i_in_kcal_angstrom"]
