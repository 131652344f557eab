"""The oracle's temperature scale, pinned by equipartition rather than by its own formula.

Velocities drawn from the Maxwell distribution at temperature T have, per Cartesian component,
variance k_B T / m; in the units used here (A/fs, g/mol, kcal/mol) that is
R T * 4.184e-4 / m with R the molar gas constant, 8.314462618 J/(mol K) (CODATA) over
4184 J/kcal.  The oracle's kinetic temperature of such a draw must come back as T within the
statistical spread of the draw; with the centre-of-mass velocity removed, equipartition over
the remaining 3N - 3 degrees of freedom gives the mean T exactly.  A wrong gas constant, a
missing 1/2, a wrong mass or unit factor or the wrong number of degrees of freedom fails one of
the two tests.
"""
import numpy as np
import pytest

import oracle as O

R_CODATA = 8.314462618 / 4184.0    # kcal/(mol K)
ACC = 4.184e-4                      # A/fs^2 per kcal/mol/A per g/mol


def maxwell(ff, types, T, rng):
    m = np.asarray(ff["mass"])[types]
    return rng.normal(size=(3, types.size)) * np.sqrt(R_CODATA * T * ACC / m)


def test_maxwell_draw_reports_its_temperature(ff):
    """2,000,000 atoms at 437 K, no rescaling: E[T] = T * 3N / (3N - 3) (the centre of mass still
    moves), relative spread sqrt(2 / (3N)) = 5.8e-4; the bound is 5 spreads."""
    rng = np.random.default_rng(20261203)
    N, T = 2_000_000, 437.0
    types = (rng.random(N) < 0.1).astype(np.uint8)   # a tenth CH3, the rest CH2
    _, Tm = O.kinetic(ff, maxwell(ff, types, T, rng), types)
    expect = T * 3 * N / (3 * N - 3)
    assert abs(Tm / expect - 1.0) < 5 * np.sqrt(2.0 / (3 * N))


def test_equipartition_after_centre_of_mass_removal(ff):
    """20,000 independent four-atom systems, each with its mass-weighted mean velocity removed:
    9 degrees of freedom remain, so the mean reported T is T itself (with 3N = 12 it would be
    3/4 of it).  The mean of chi^2_9 / 9 has relative spread sqrt(2 / 9 / 20000) = 3.3e-3."""
    rng = np.random.default_rng(7)
    K, n, T = 20_000, 4, 310.0
    types = np.array([1, 0, 0, 1], dtype=np.uint8)
    m = np.asarray(ff["mass"])[types]
    Ts = np.empty(K)
    for k in range(K):
        v = maxwell(ff, types, T, rng)
        v -= (v * m).sum(axis=1, keepdims=True) / m.sum()
        Ts[k] = O.kinetic(ff, v, types)[1]
    assert abs(Ts.mean() / T - 1.0) < 5 * np.sqrt(2.0 / 9.0 / K)
