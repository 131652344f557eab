"""Pins of the oracle's bond, angle and dihedral terms (Eqs. 4-6, Section 3.3)."""
import numpy as np
import pytest

import oracle as O


def _rot(axis, ang):
    axis = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + np.sin(ang) * K + (1 - np.cos(ang)) * K @ K


def _dihedral_geometry(phi_deg):
    """i-j-k-l with j at the origin, k on +x, i on +y; l's bond rotated clockwise by phi (seen
    from j looking at k, screen right = +z), i.e. IUPAC phi."""
    p = np.deg2rad(phi_deg)
    return (np.array([0.0, 1.0, 0.0]), np.zeros(3), np.array([1.0, 0.0, 0.0]),
            np.array([1.0, np.cos(p), np.sin(p)]))


def test_bond_closed_form(ff):
    for delta in (0.0, 0.01, -0.03, 0.2):
        xi = np.array([1.0, 2.0, 3.0])
        u = np.array([0.3, -0.5, 0.8]) / np.linalg.norm([0.3, -0.5, 0.8])
        xj = xi + (ff["b0"] + delta) * u
        e, f = O.bond_term(ff, xi, xj)
        assert e == pytest.approx(0.5 * ff["kb"] * delta ** 2, rel=1e-11, abs=1e-24)
        # stretched bond pulls the atoms together with magnitude kb*delta
        np.testing.assert_allclose(f[0], ff["kb"] * delta * u, rtol=1e-11, atol=1e-11)
        np.testing.assert_allclose(f[1], -f[0], rtol=0, atol=0)


@pytest.mark.parametrize("dtheta_deg", [0.0, 5.0, -12.0, 30.0])
def test_angle_closed_form(ff, dtheta_deg):
    th = np.deg2rad(ff["theta0_deg"] + dtheta_deg)
    xj = np.array([0.5, -1.0, 2.0])
    xi = xj + 1.53 * np.array([1.0, 0.0, 0.0])
    xk = xj + 1.7 * np.array([np.cos(th), np.sin(th), 0.0])
    e, f, theta = O.angle_term(ff, xi, xj, xk)
    assert theta == pytest.approx(th, abs=1e-14)
    assert e == pytest.approx(0.5 * ff["ka"] * np.deg2rad(dtheta_deg) ** 2, rel=1e-11, abs=1e-28)


@pytest.mark.parametrize("phi,expect", [(180.0, 0.0), (60.0, 0.0), (-60.0, 0.0), (0.0, 2.0),
                                        (90.0, 1.0), (-90.0, 1.0), (120.0, 2.0), (30.0, 1.0)])
def test_dihedral_closed_form(ff, phi, expect):
    e, f, ph = O.dihedral_term(ff, *_dihedral_geometry(phi))
    assert e == pytest.approx(expect * ff["kphi"], abs=1e-14)
    d = (np.rad2deg(ph) - phi + 180.0) % 360.0 - 180.0
    assert abs(d) < 1e-11                          # IUPAC sign, trans = 180


def test_dihedral_sign_convention(ff):
    """IUPAC: positive when the front bond turns clockwise onto the back bond."""
    _, _, ph = O.dihedral_term(ff, *_dihedral_geometry(90.0))
    assert ph == pytest.approx(np.pi / 2, abs=1e-14)
    _, _, ph = O.dihedral_term(ff, *_dihedral_geometry(-90.0))
    assert ph == pytest.approx(-np.pi / 2, abs=1e-14)


def _fd_check(fun, coords, h=1e-5, rel=1e-6):
    e0, f = fun(*coords)[:2]
    for a in range(len(coords)):
        for d in range(3):
            cp = [c.copy() for c in coords]
            cm = [c.copy() for c in coords]
            cp[a][d] += h
            cm[a][d] -= h
            fd = -(fun(*cp)[0] - fun(*cm)[0]) / (2 * h)
            assert fd == pytest.approx(f[a, d], rel=rel, abs=1e-7)
    return f


def _invariants(f, coords):
    assert np.abs(f.sum(axis=0)).max() < 1e-11 * (1 + np.abs(f).max())
    torque = sum(np.cross(c, fa) for c, fa in zip(coords, f))
    assert np.abs(torque).max() < 1e-10 * (1 + np.abs(f).max())


def test_bonded_finite_differences_and_invariants(ff):
    rng = np.random.default_rng(3)
    for _ in range(20):
        base = [np.zeros(3)]
        for _k in range(3):
            base.append(base[-1] + rng.normal(size=3))
        c = [b + rng.normal(scale=0.1, size=3) for b in base]
        f = _fd_check(lambda a, b: O.bond_term(ff, a, b), c[:2])
        _invariants(f, c[:2])
        f = _fd_check(lambda a, b, d: O.angle_term(ff, a, b, d)[:2], c[:3])
        _invariants(f, c[:3])
        f = _fd_check(lambda a, b, d, g: O.dihedral_term(ff, a, b, d, g)[:2], c[:4])
        _invariants(f, c[:4])
        # generalised dihedral: n = 2, phi_s = 30 deg
        ff2 = dict(ff, n_dih=2, phis_deg=30.0)
        f = _fd_check(lambda a, b, d, g: O.dihedral_term(ff2, a, b, d, g)[:2], c[:4])
        _invariants(f, c[:4])


def test_bonded_rigid_motion_invariance(ff):
    rng = np.random.default_rng(4)
    c = [rng.normal(size=3) * 1.5 for _ in range(4)]
    R = _rot([1.0, 2.0, -0.5], 0.7)
    t = np.array([3.0, -2.0, 1.0])
    e0, f0, _ = O.dihedral_term(ff, *c)
    e1, f1, _ = O.dihedral_term(ff, *[R @ x + t for x in c])
    assert e1 == pytest.approx(e0, rel=1e-12)
    np.testing.assert_allclose(f1, (R @ f0.T).T, rtol=1e-9, atol=1e-12)
    e0, f0, _ = O.angle_term(ff, *c[:3])
    e1, f1, _ = O.angle_term(ff, *[R @ x + t for x in c[:3]])
    assert e1 == pytest.approx(e0, rel=1e-12)
    np.testing.assert_allclose(f1, (R @ f0.T).T, rtol=1e-9, atol=1e-12)


def test_chain_bonded_sums_terms_and_respects_periodicity(ff, melt3k):
    m = melt3k
    f, e = O.bonded(ff, m.pos, m.box, 300)
    assert np.abs(f.sum(axis=1)).max() < 1e-10 * np.abs(f).sum()
    # chain 0 term by term, on unwrapped coordinates
    from pe_melt import unwrap_chains
    u = unwrap_chains(m.pos, m.box, 300)[:, :300].T
    fe = np.zeros((300, 3))
    eb = ea = ed = 0.0
    for (i, j) in O.chain_terms(300, 2):
        en, ft = O.bond_term(ff, u[i], u[j]); eb += en; fe[[i, j]] += ft
    for (i, j, k) in O.chain_terms(300, 3):
        en, ft, _ = O.angle_term(ff, u[i], u[j], u[k]); ea += en; fe[[i, j, k]] += ft
    for (i, j, k, l) in O.chain_terms(300, 4):
        en, ft, _ = O.dihedral_term(ff, u[i], u[j], u[k], u[l]); ed += en; fe[[i, j, k, l]] += ft
    np.testing.assert_allclose(f[:, :300].T, fe, rtol=1e-9, atol=1e-9)
    # the whole box in a box large enough that nothing wraps gives the same answer
    big = np.array([1e4] * 3)
    uw = unwrap_chains(m.pos, m.box, 300) + 5e3
    f2, e2 = O.bonded(ff, uw, big, 300)
    np.testing.assert_allclose(f2, f, rtol=1e-8, atol=1e-8)
    for k in ("e_bond", "e_angle", "e_dih"):
        assert e2[k] == pytest.approx(e[k], rel=1e-10)
