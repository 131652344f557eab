"""Input data: Table I conversions, melt geometry and velocities."""
import numpy as np
import pytest

import oracle as O
from pe_melt import WORKLOADS, box_length, make_melt, polyethylene_forcefield, table_i_in_kcal_angstrom
from pe_melt.generator import ACC_UNIT, R_KCAL


def test_table_i_conversion():
    """Table I (kJ/mol, nm) in kcal/mol and Angstrom: 292880 kJ/mol/nm^2 = 700 kcal/mol/A^2,
    418.40 kJ/mol/rad^2 = 100 kcal/mol/rad^2, 4.184 kJ/mol = 1 kcal/mol, 0.153 nm = 1.53 A."""
    t = table_i_in_kcal_angstrom()
    assert t["kb"] == pytest.approx(700.0, rel=1e-14)
    assert t["ka"] == pytest.approx(100.0, rel=1e-14)
    assert t["kphi"] == pytest.approx(1.0, rel=1e-14)
    assert t["b0"] == pytest.approx(1.53, rel=1e-14)
    assert t["theta0_deg"] == 109.471
    assert t["n_dih"] == 3 and t["phis_deg"] == 0.0
    ff = polyethylene_forcefield()
    assert ff["mass"] == (14.027, 15.035)
    # united-atom masses: C + 2H and C + 3H
    assert ff["mass"][0] == pytest.approx(12.011 + 2 * 1.008, abs=1e-9)
    assert ff["mass"][1] == pytest.approx(12.011 + 3 * 1.008, abs=1e-9)
    assert ff["excl_depth"] == 2


@pytest.mark.parametrize("chains,rho,L", [(10, 0.80, 44.376), (1000, 0.80, 205.977),
                                          (10000, 0.85, 434.885), (100000, 0.85, 936.932)])
def test_box_sizes(chains, rho, L):
    assert box_length(chains, 300, rho) == pytest.approx(L, abs=2e-3)


def test_workload_presets():
    assert WORKLOADS["melt3k_fp64"].n_atoms == 3000
    assert WORKLOADS["melt300k_mixed"].n_atoms == 300_000
    assert WORKLOADS["melt3M_mixed"].n_atoms == 3_000_000
    ens = WORKLOADS["ensemble64_mixed"]
    assert ens.n_boxes == 64 and min(ens.n_chains) >= 20 and max(ens.n_chains) <= 400
    assert ens.T0[0] == 250.0 and ens.T0[-1] == 450.0


def test_melt_geometry_and_velocities(ff):
    m = make_melt(10, seed_melt=1000, seed_vel=1001)
    N = m.n_atoms
    assert N == 3000 and m.pos.shape == (3, N)
    assert np.all(m.pos >= 0) and np.all(m.pos < m.box[:, None])
    assert m.types[0] == 1 and m.types[299] == 1 and m.types[1:299].max() == 0
    # bonds exact, angles at 109.47, bonded energy ~0 (trans and gauche are minima of Eq. 6)
    f, e = O.bonded(ff, m.pos, m.box, 300)
    assert e["e_bond"] < 1e-18 * N
    # the grower's 109.47 deg sits 0.001 deg off theta0 = 109.471 deg
    n_angles = 10 * 298
    assert e["e_angle"] == pytest.approx(n_angles * 0.5 * 100.0 * np.deg2rad(0.001) ** 2, rel=1e-3)
    # velocities: zero momentum, exact temperature with 3N-3 dof
    mass = np.asarray(ff["mass"])[m.types]
    assert np.abs((m.vel * mass).sum(axis=1)).max() < 1e-10
    ke, T = O.kinetic(ff, m.vel, m.types)
    assert T == pytest.approx(500.0, rel=1e-12)
    assert ke == pytest.approx(0.5 * np.sum(mass * m.vel ** 2) / ACC_UNIT, rel=1e-12)
    assert R_KCAL == 1.987204259e-3


def test_melt_clearance_and_determinism():
    from scipy.spatial import cKDTree
    a = make_melt(10, seed_melt=1000)
    b = make_melt(10, seed_melt=1000)
    assert np.array_equal(a.pos, b.pos) and np.array_equal(a.vel, b.vel)
    p = a.pos.T
    pairs = cKDTree(p, boxsize=a.box[0] + 1e-9).query_pairs(2.0, output_type="ndarray")
    i, j = pairs[:, 0], pairs[:, 1]
    nonlocal_ = (i // 300 != j // 300) | (np.abs(i - j) > 3)
    assert not nonlocal_.any()


def test_tiled_melt_copies_the_small_melt():
    """tiles^3 copies of a small melt: bonds intact across the copy faces, the large box holds
    the same density, and every atom's nearest non-bonded neighbour is the one it had in the
    small periodic box."""
    from scipy.spatial import cKDTree

    from pe_melt import box_length, make_melt, make_tiled_melt, unwrap_chains
    small = make_melt(10, density=0.85, T=300.0, seed_melt=31, seed_vel=32)
    big = make_tiled_melt(80, 2, density=0.85, T=300.0, seed_melt=31, seed_vel=32)
    assert big.n_atoms == 8 * small.n_atoms
    assert np.allclose(big.box, 2 * small.box) and big.box[0] == pytest.approx(box_length(80, 300, 0.85), rel=1e-12)
    u = unwrap_chains(big.pos, big.box, 300).T.reshape(-1, 300, 3)
    b = np.sqrt(np.sum(np.diff(u, axis=1) ** 2, axis=-1))
    assert np.allclose(b, 1.53, atol=1e-9)
    assert np.all((big.pos >= 0) & (big.pos < big.box[:, None]))

    def nearest(m):
        t = cKDTree(m.pos.T, boxsize=m.box)
        d, _ = t.query(m.pos.T, k=2)
        return np.sort(d[:, 1])
    ds, db = nearest(small), nearest(big)
    np.testing.assert_allclose(db[::8], ds, rtol=0, atol=1e-9)
    # velocities are drawn for the whole system, not copied
    assert not np.allclose(big.vel[:, :small.n_atoms], big.vel[:, small.n_atoms:2 * small.n_atoms])
