"""Pins of the oracle's Section 5 observables: the pair-distance histogram behind the radial
distribution function (Fig. 10), the dihedral statistics behind the conformation
distribution and the trans fraction (Figs. 9, 15), and the chain shape (R_g, Fig. 12;
end-to-end vector, Fig. 8).

What fixes them, other than the oracle itself: the coordination shells of a simple cubic
lattice; brute force against the grid search; the 1-2 and 1-3 pairs the exclusions remove,
from the chain geometry; the ideal-gas shell volumes; chains built from prescribed internal
coordinates; the closed forms of a straight rod and of the planar all-trans zigzag.
"""
import math

import numpy as np
import pytest

import oracle as O

A = 4.03   # lattice spacing, A: every shell distance lies well inside a 0.1 A bin


def lattice(n=8, a=A):
    g = np.arange(n) * a + 0.5
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()]), np.full(3, n * a)


def test_simple_cubic_shells():
    """Shells of a simple cubic lattice at a sqrt(k): 6, 12, 8, 6, 24, 24 neighbours per atom
    for k = 1..6; each unordered pair once."""
    pos, box = lattice()
    n = pos.shape[1]
    rmax, bins = 10.0, 100
    expected = np.zeros(bins, dtype=np.uint64)
    for k, z in zip(range(1, 7), (6, 12, 8, 6, 24, 24)):
        expected[int(A * math.sqrt(k) / 0.1)] += n * z // 2
    for cells in (False, True):
        h = O.pair_histogram(pos, box, 1, 2, rmax, bins, cells=cells)
        np.testing.assert_array_equal(h, expected)


def test_grid_search_equals_brute_force(melt3k):
    m = melt3k
    for rmax, bins in ((10.5, 105), (7.0, 350)):
        a = O.pair_histogram(m.pos, m.box, 300, 2, rmax, bins, cells=True)
        b = O.pair_histogram(m.pos, m.box, 300, 2, rmax, bins, cells=False)
        np.testing.assert_array_equal(a, b)
        assert a.sum() > 0


def test_exclusions_remove_exactly_the_1_2_and_1_3_pairs(melt3k):
    m = melt3k
    rmax, bins = 10.5, 210
    diff = (O.pair_histogram(m.pos, m.box, 300, 0, rmax, bins).astype(np.int64)
            - O.pair_histogram(m.pos, m.box, 300, 2, rmax, bins).astype(np.int64))
    expected = np.zeros(bins, dtype=np.int64)
    for c in range(m.n_chains):
        for step in (1, 2):
            i = np.arange(c * 300, (c + 1) * 300 - step)
            d = m.pos[:, i] - m.pos[:, i + step]
            d -= m.box[:, None] * np.round(d / m.box[:, None])
            r = np.sqrt(np.sum(d * d, axis=0))
            np.add.at(expected, (r / (rmax / bins)).astype(int), 1)
    assert expected.sum() == m.n_chains * (299 + 298)
    np.testing.assert_array_equal(diff, expected)


def test_ideal_gas_shell_counts():
    """Uniform points: the pairs in each shell follow N(N-1)/2 * shell volume / V."""
    rng = np.random.default_rng(3)
    L, n = 30.0, 3000
    pos = rng.random((3, n)) * L
    rmax, bins = 10.0, 20
    h = O.pair_histogram(pos, [L] * 3, 1, 2, rmax, bins).astype(float)
    edges = np.arange(bins + 1) * (rmax / bins)
    ideal = n * (n - 1) / 2 * (4 / 3 * np.pi * (edges[1:] ** 3 - edges[:-1] ** 3)) / L ** 3
    assert abs(h.sum() / ideal.sum() - 1) < 0.01
    z = (h - ideal) / np.sqrt(ideal)
    assert np.all(np.abs(z[4:]) < 5.0)


def build_chain(dihedrals_deg, b=1.53, theta_deg=109.471, origin=(3.0, 4.0, 5.0)):
    """Chain from internal coordinates: every bond b, every angle theta, and the listed
    dihedral angles (i, i+1, i+2, i+3) in the IUPAC sense (trans = 180)."""
    th = math.radians(theta_deg)
    x = [np.array(origin), np.array(origin) + [b, 0, 0],
         np.array(origin) + [b - b * math.cos(th), b * math.sin(th), 0]]
    for phi_deg in dihedrals_deg:
        a, bb, c = x[-3], x[-2], x[-1]
        bc = (c - bb) / np.linalg.norm(c - bb)
        nrm = np.cross(bb - a, bc)
        nrm /= np.linalg.norm(nrm)
        mm = np.cross(nrm, bc)
        phi = math.radians(phi_deg)
        d2 = np.array([-b * math.cos(th), b * math.sin(th) * math.cos(phi), b * math.sin(th) * math.sin(phi)])
        x.append(c + d2[0] * bc + d2[1] * mm + d2[2] * nrm)
    return np.array(x).T


def test_dihedral_classes_and_histogram_of_a_built_chain(ff):
    phis = [180, 60, -60, 175, 75, -100, 150, -170, 10, -10, 119, -119, 121, -121, 179.5, -45, 90, -150]
    pos = build_chain(phis)
    n = pos.shape[1]
    # the angle the force field computes is the prescribed one (IUPAC, sign included)
    for t, phi in enumerate(phis):
        _, _, got = O.dihedral_term(ff, pos[:, t], pos[:, t + 1], pos[:, t + 2], pos[:, t + 3])
        d = (math.degrees(got) - phi + 180) % 360 - 180
        assert abs(d) < 1e-9
    box = np.array([200.0, 200.0, 200.0])
    # 7 bins of 360/7 deg: no prescribed angle lies near an edge
    hist, cls = O.dihedral_stats(pos, box, n, 7)
    expect_hist = np.zeros(7, dtype=np.uint64)
    for phi in phis:
        expect_hist[min(int((phi + 180) // (360 / 7)), 6)] += 1
    np.testing.assert_array_equal(hist, expect_hist)
    trans = sum(abs(p) > 120 for p in phis)
    gplus = sum(0 <= p <= 120 for p in phis)
    np.testing.assert_array_equal(cls, [trans, gplus, len(phis) - trans - gplus])


def test_dihedral_stats_are_periodic(ff):
    """The same chain moved across the box faces and wrapped: unchanged statistics."""
    phis = list(np.random.default_rng(1).uniform(-179, 179, 40))
    pos = build_chain(phis)
    box = np.array([15.0, 15.0, 15.0])
    moved = O.wrap(pos + np.array([[13.0], [-7.5], [29.0]]), box)
    for n_bins in (0, 24):
        h1, c1 = O.dihedral_stats(pos, [500.0] * 3, pos.shape[1], n_bins)
        h2, c2 = O.dihedral_stats(moved, box, pos.shape[1], n_bins)
        np.testing.assert_array_equal(h1, h2)
        np.testing.assert_array_equal(c1, c2)


def test_rod_and_zigzag_closed_forms(ff):
    """Equal masses: a straight rod of n atoms at spacing b has Rg^2 = b^2 (n^2 - 1) / 12 and
    R_ee = (n - 1) b; the planar all-trans zigzag advances b sin(theta/2) per bond along its
    axis and ends b cos(theta/2) off it when n is even."""
    f = dict(ff)
    f["mass"] = (14.027, 14.027)
    n, b = 300, 1.53
    types = np.zeros(n, np.uint8)
    types[[0, -1]] = 1
    rod = np.stack([np.arange(n) * b, np.full(n, 2.0), np.full(n, 3.0)])
    box = np.array([40.0, 40.0, 40.0])
    out = O.chain_shape(f, O.wrap(rod, box), types, box, n)   # 459 A rod in a 40 A box
    assert out[0, 0] == pytest.approx(b * b * (n * n - 1) / 12, rel=1e-12)
    np.testing.assert_allclose(out[0, 1:], [(n - 1) * b, 0, 0], atol=1e-9)
    th = math.radians(109.471)
    zz = build_chain([180.0] * (n - 3), b=b, theta_deg=109.471)
    out = O.chain_shape(f, O.wrap(zz, box), types, box, n)
    ree = np.linalg.norm(out[0, 1:])
    along, off = (n - 1) * b * math.sin(th / 2), b * math.cos(th / 2)
    assert ree == pytest.approx(math.hypot(along, off), rel=1e-10)


def test_chain_shape_is_translation_invariant_and_mass_weighted(ff, melt3k):
    m = melt3k
    a = O.chain_shape(ff, m.pos, m.types, m.box, 300)
    b = O.chain_shape(ff, O.wrap(m.pos + np.array([[17.3], [-41.0], [5.5]]), m.box), m.types, m.box, 300)
    np.testing.assert_allclose(a, b, rtol=1e-10, atol=1e-9)
    # the masses weight R_g but not the end-to-end vector
    f = dict(ff)
    f["mass"] = (14.027, 14.027)
    c = O.chain_shape(f, m.pos, m.types, m.box, 300)
    assert np.all(a[:, 0] != c[:, 0])
    np.testing.assert_allclose(a[:, 1:], c[:, 1:], rtol=0, atol=0)


def test_mass_weighted_rod(ff):
    """A straight rod with heavier CH3 ends: the centre of mass stays at the middle, and
    Rg^2 = b^2 [m (n (n^2 - 1) / 12 - 2 c^2) + 2 M c^2] / (m (n - 2) + 2 M), c = (n - 1) / 2."""
    n, b = 300, 1.53
    m, M = ff["mass"]
    types = np.zeros(n, np.uint8)
    types[[0, -1]] = 1
    rod = np.stack([np.full(n, 2.0), np.arange(n) * b, np.full(n, 3.0)])
    box = np.array([40.0, 40.0, 40.0])
    out = O.chain_shape(ff, O.wrap(rod, box), types, box, n)
    c = (n - 1) / 2
    rg2 = b * b * (m * (n * (n * n - 1) / 12 - 2 * c * c) + 2 * M * c * c) / (m * (n - 2) + 2 * M)
    assert out[0, 0] == pytest.approx(rg2, rel=1e-12)


def _rotate(u, axis, theta):
    """Rodrigues rotation of the points u [3, n] about the unit axis through their first point."""
    k = np.asarray(axis, dtype=float) / np.linalg.norm(axis)
    p = u - u[:, :1]
    c, s = math.cos(theta), math.sin(theta)
    rot = p * c + np.cross(k, p.T).T * s + np.outer(k, k @ p) * (1.0 - c)
    return rot + u[:, :1]


def test_end_to_end_acf_closed_forms(melt3k):
    """Fig. 8's end-to-end autocorrelation: 1 for the reference itself and after a rigid
    translation (any wrap); cos(theta) when every chain is turned rigidly by theta about an axis
    perpendicular to its end-to-end vector; -1 when every chain is point-reflected; and for
    chains turned by different angles, the |R|^2-weighted mean of the cosines."""
    from pe_melt import unwrap_chains
    m = melt3k
    L, n = m.box, m.chain_len
    assert O.ree_acf(m.pos, m.pos, L, n) == pytest.approx(1.0, abs=1e-15)
    shifted = np.mod(m.pos + np.array([[17.3], [-101.9], [4.4]]), L[:, None])
    assert O.ree_acf(m.pos, shifted, L, n) == pytest.approx(1.0, abs=1e-13)
    u = unwrap_chains(m.pos, L, n)
    chains = [u[:, c * n:(c + 1) * n] for c in range(m.n_chains)]
    ree = np.array([ch[:, -1] - ch[:, 0] for ch in chains])
    rng = np.random.default_rng(3)

    def turned(thetas):
        out = []
        for ch, r, th in zip(chains, ree, thetas):
            axis = np.cross(r, rng.normal(size=3))       # perpendicular to this chain's R
            out.append(_rotate(ch, axis, th))
        return np.mod(np.concatenate(out, axis=1), L[:, None])

    for theta in (0.3, 1.1, math.pi / 2, 2.5):
        assert O.ree_acf(m.pos, turned([theta] * m.n_chains), L, n) == pytest.approx(math.cos(theta), abs=1e-12)
    reflected = np.mod(np.concatenate([2 * ch[:, :1] - ch for ch in chains], axis=1), L[:, None])
    assert O.ree_acf(m.pos, reflected, L, n) == pytest.approx(-1.0, abs=1e-13)
    thetas = rng.uniform(0, math.pi, size=m.n_chains)
    w = np.sum(ree ** 2, axis=1)
    assert O.ree_acf(m.pos, turned(thetas), L, n) == pytest.approx(np.sum(w * np.cos(thetas)) / w.sum(), abs=1e-12)
