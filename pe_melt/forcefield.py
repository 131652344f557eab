"""Force-field parameters for united-atom polyethylene, as plain input data.

Source: the paper's Table I (Dreiding II subset for the C_32 = CH2 and C_33 = CH3
united atoms) and Eqs. (2)-(6).  The table's header is garbled in the text we
have; the reading used here:

* The first numeric column of the atom rows (14.027 / 15.035) is the united-atom
  mass in g/mol (12.011 + 2*1.008 and + 3*1.008), not sigma.  Only one LJ number
  per type survives, so the Lennard-Jones sigma/epsilon pair comes from the melt
  recipe instead: sigma = 3.47 A, epsilon = 0.0951 kcal/mol for both types.
* Bond constant 292880 kJ/mol/nm^2 and length 0.153 nm; angle constant
  418.40 kJ/mol/rad^2 and 109.471 deg; dihedral 4.184 kJ/mol, phi_s = 0, n = 3.
  Eqs. (4) and (5) carry the factor 1/2.

This module only converts units (kJ -> kcal by the thermochemical 4.184, nm -> A);
it holds none of the simulation arithmetic and is shared, as input data, by the
CPU reference and the GPU library.
"""

from __future__ import annotations

KJ_PER_KCAL = 4.184          # thermochemical calorie
A_PER_NM = 10.0

# Table I, as printed (SI-ish units of the paper)
TABLE_I = {
    "mass": {"C_32": 14.027, "C_33": 15.035},           # g/mol (see reading above)
    "bond_k_kj_nm2": 292880.0, "bond_b_nm": 0.153,
    "angle_k_kj_rad2": 418.40, "angle_theta0_deg": 109.471,
    "dihedral_k_kj": 4.184, "dihedral_phis_deg": 0.0, "dihedral_n": 3,
}

# Lennard-Jones pair from the melt recipe (Table I's LJ columns are unrecoverable)
LJ_SIGMA_A = 3.47
LJ_EPSILON_KCAL = 0.0951
R_CUT_A = 10.5


def table_i_in_kcal_angstrom() -> dict:
    """Table I converted to kcal/mol, Angstrom, radian/degree units."""
    t = TABLE_I
    return {
        "kb": t["bond_k_kj_nm2"] / KJ_PER_KCAL / (A_PER_NM ** 2),     # kcal/mol/A^2
        "b0": t["bond_b_nm"] * A_PER_NM,                               # A
        "ka": t["angle_k_kj_rad2"] / KJ_PER_KCAL,                      # kcal/mol/rad^2
        "theta0_deg": t["angle_theta0_deg"],
        "kphi": t["dihedral_k_kj"] / KJ_PER_KCAL,                      # kcal/mol
        "phis_deg": t["dihedral_phis_deg"],
        "n_dih": t["dihedral_n"],
    }


def polyethylene_forcefield(rc: float = R_CUT_A) -> dict:
    """The parameter set every configuration uses (keys mirror ``md_forcefield``)."""
    b = table_i_in_kcal_angstrom()
    return {
        "mass": (TABLE_I["mass"]["C_32"], TABLE_I["mass"]["C_33"]),
        "sigma": (LJ_SIGMA_A, LJ_SIGMA_A),
        "epsilon": (LJ_EPSILON_KCAL, LJ_EPSILON_KCAL),
        "kb": b["kb"], "b0": b["b0"],
        "ka": b["ka"], "theta0_deg": b["theta0_deg"],
        "kphi": b["kphi"], "phis_deg": b["phis_deg"], "n_dih": b["n_dih"],
        "rc": rc,
        "excl_depth": 2,   # Dreiding II: only 1-2 and 1-3 neighbours are excluded
    }
