"""Pins of the oracle's Lennard-Jones term (Eq. 2, Section 3.2)."""
import numpy as np
import pytest

import oracle as O


def _two_atoms(r, box=40.0):
    pos = np.array([[5.0, 5.0 + r], [7.0, 7.0], [9.0, 9.0]])
    return pos, np.zeros(2, np.uint8), np.array([box] * 3)


def test_lj_special_values(ff):
    sig, eps, rc = ff["sigma"][0], ff["epsilon"][0], ff["rc"]
    # chain_len 1: two independent atoms, never excluded
    f, e = O.lj_brute(ff, *_two_atoms(sig), 1)
    assert abs(e["e_lj"]) < 1e-15                                   # E(sigma) = 0
    rmin = 2 ** (1 / 6) * sig
    f, e = O.lj_brute(ff, *_two_atoms(rmin), 1)
    assert e["e_lj"] == pytest.approx(-eps, rel=1e-13)              # E(r_min) = -eps
    assert np.abs(f).max() < 1e-13                                  # and zero force there
    f, e = O.lj_brute(ff, *_two_atoms(np.nextafter(rc, 0)), 1)
    assert e["e_lj"] < 0 and np.abs(f[0]).max() > 0                 # just inside rc: counted
    f, e = O.lj_brute(ff, *_two_atoms(rc), 1)
    assert e["e_lj"] == 0.0 and np.abs(f).max() == 0.0              # at rc: strict cutoff
    # shifted energy is zero at the cutoff end and E(r) - E(rc) inside
    r = 5.0
    f, e = O.lj_brute(ff, *_two_atoms(r), 1)
    assert e["e_lj_shifted"] - e["e_lj"] == pytest.approx(-(4 * eps * ((sig / rc) ** 12 - (sig / rc) ** 6)),
                                                          rel=1e-12)
    # far tail: E ~ -4 eps (sigma/r)^6 within the (sigma/r)^6 correction
    f, e = O.lj_brute(ff, *_two_atoms(10.0), 1)
    tail = -4 * eps * (sig / 10.0) ** 6
    assert e["e_lj"] == pytest.approx(tail, rel=2 * (sig / 10.0) ** 6)
    # repulsive inside r_min: force pushes atom 0 away from atom 1 (atom 1 is at +x)
    f, e = O.lj_brute(ff, *_two_atoms(3.2), 1)
    assert f[0, 0] < 0 < f[0, 1]
    # virial of one pair = F_ij . r_ij
    assert e["virial_lj"] == pytest.approx(-f[0, 0] * 3.2, rel=1e-13)


def test_lj_energy_scales_with_sigma_and_epsilon(ff):
    r = 4.1
    _, e1 = O.lj_brute(ff, *_two_atoms(r), 1)
    ff2 = dict(ff, sigma=(2 * ff["sigma"][0],) * 2, epsilon=(3 * ff["epsilon"][0],) * 2, rc=2 * ff["rc"])
    _, e2 = O.lj_brute(ff2, *_two_atoms(2 * r, box=90.0), 1)
    assert e2["e_lj"] == pytest.approx(3 * e1["e_lj"], rel=1e-13)


def test_lj_finite_difference(ff):
    rng = np.random.default_rng(11)
    n, L = 60, 32.0
    pos = rng.random((3, n)) * L
    types = rng.integers(0, 2, n).astype(np.uint8)
    ffm = dict(ff, sigma=(3.47, 3.6), epsilon=(0.0951, 0.12))
    f, _ = O.lj_brute(ffm, pos, types, [L] * 3, 1)
    h = 1e-5
    for i in rng.choice(n, 8, replace=False):
        for d in range(3):
            p1, p2 = pos.copy(), pos.copy()
            p1[d, i] += h
            p2[d, i] -= h
            e1 = O.lj_brute(ffm, p1, types, [L] * 3, 1)[1]["e_lj"]
            e2 = O.lj_brute(ffm, p2, types, [L] * 3, 1)[1]["e_lj"]
            fd = -(e1 - e2) / (2 * h)
            assert fd == pytest.approx(f[d, i], rel=1e-6, abs=1e-7)


def test_lj_exclusions_1_2_and_1_3_only(ff):
    # one 4-site chain, straight, in a large box: only the 1-4 pair interacts
    pos = np.array([[5.0, 6.53, 8.06, 9.59], [5.0] * 4, [5.0] * 4])
    f, e = O.lj_brute(ff, pos, np.zeros(4, np.uint8), [40.0] * 3, 4)
    f14, e14 = O.lj_brute(ff, pos[:, [0, 3]], np.zeros(2, np.uint8), [40.0] * 3, 1)
    assert e["e_lj"] == pytest.approx(e14["e_lj"], rel=1e-15) and e["e_lj"] != 0
    np.testing.assert_allclose(f[:, [0, 3]], f14, rtol=1e-15)
    assert np.all(f[:, [1, 2]] == 0)
    # the same four atoms as separate molecules: every pair interacts
    f_free, e_free = O.lj_brute(ff, pos, np.zeros(4, np.uint8), [40.0] * 3, 1)
    assert e_free["e_lj"] > 1e3


def test_lj_brute_equals_grid_search(ff, melt3k):
    m = melt3k
    fb, eb = O.lj_brute(ff, m.pos, m.types, m.box, 300)
    for R in (1, 2):
        fc, ec = O.lj_cells(ff, m.pos, m.types, m.box, 300, R=R)
        scale = np.abs(fb).max()
        assert np.abs(fb - fc).max() <= 1e-12 * scale
        for k in ("e_lj", "e_lj_shifted", "virial_lj"):
            assert ec[k] == pytest.approx(eb[k], rel=1e-12)
    # Newton's third law
    assert np.abs(fb.sum(axis=1)).max() <= 1e-11 * np.abs(fb).sum()
    # a subset evaluation reproduces the same rows
    sub = np.array([0, 1, 299, 1500, 2999])
    fs, _ = O.lj_cells(ff, m.pos, m.types, m.box, 300, subset=sub)
    assert np.abs(fs - fb[:, sub]).max() <= 1e-12 * np.abs(fb).max()


def test_lj_translation_invariance(ff, melt3k):
    m = melt3k
    f0, e0 = O.lj_cells(ff, m.pos, m.types, m.box, 300)
    shifted = O.wrap(m.pos + np.array([[3.3], [-17.1], [40.2]]), m.box)
    f1, e1 = O.lj_cells(ff, shifted, m.types, m.box, 300)
    assert e1["e_lj"] == pytest.approx(e0["e_lj"], rel=1e-11)
    assert np.abs(f1 - f0).max() <= 1e-9 * np.abs(f0).max()


def test_lj_rejects_bad_grid(ff, melt3k):
    m = melt3k
    with pytest.raises(RuntimeError):
        O.lj_cells(ff, m.pos, m.types, m.box, 300, M=np.array([2, 4, 4], np.int32))    # M < 3
    with pytest.raises(RuntimeError):
        O.lj_cells(ff, m.pos, m.types, m.box, 300, M=np.array([5, 4, 4], np.int32))    # edge < rc
    bad = m.pos.copy()
    bad[0, 0] = -1.0
    with pytest.raises(RuntimeError):
        O.lj_cells(ff, bad, m.types, m.box, 300)                                        # not wrapped
