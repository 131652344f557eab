"""Pins of the oracle's wrap, cell index and counting sort (Section 3.1)."""
import numpy as np
import pytest

import oracle as O


def _boundary_positions(L, M, rng, n_random=4000):
    """Random points plus exact cell faces, 0, and the largest double below L."""
    faces = np.concatenate([np.arange(M) * (L / M), [0.0, np.nextafter(L, 0.0)]])
    pts = []
    for d in range(3):
        col = rng.random(n_random + faces.size) * L
        col[:faces.size] = np.roll(faces, d)
        pts.append(col)
    return np.array(pts)


@pytest.mark.parametrize("M", [3, 4, 7])
def test_cell_index_bounds(M):
    rng = np.random.default_rng(5)
    L = np.array([44.376, 37.1, 52.9])
    pos = np.stack([_boundary_positions(L[d], M, rng)[d] for d in range(3)])
    Mv = np.array([M, M + 1, M + 2], dtype=np.int32)
    cell = O.cell_index(pos, L, Mv)
    k = np.stack([cell % Mv[0], (cell // Mv[0]) % Mv[1], cell // (Mv[0] * Mv[1])])
    assert k.min() >= 0 and np.all(k < Mv[:, None])
    edge = L / Mv
    # every atom lies inside its cell (up to the rounding of x * M / L)
    lo = k * edge[:, None]
    hi = (k + 1) * edge[:, None]
    tol = 4 * np.finfo(float).eps * L[:, None]
    assert np.all(pos >= lo - tol) and np.all(pos < hi + tol)
    # points exactly on a face go to the upper cell; 0 -> 0; just below L -> M-1
    assert k[0][pos[0] == 0.0].max() == 0
    assert np.all(k[0][pos[0] == np.nextafter(L[0], 0.0)] == Mv[0] - 1)


def test_bin_is_stable_counting_sort():
    rng = np.random.default_rng(6)
    n, n_cells = 5000, 64
    cell = rng.integers(0, n_cells, size=n).astype(np.int32)
    cnt, start, atoms = O.bin_atoms(cell, n_cells)
    assert cnt.sum() == n and start[0] == 0 and start[-1] == n
    np.testing.assert_array_equal(np.diff(start), cnt)
    np.testing.assert_array_equal(np.sort(atoms), np.arange(n))          # a permutation
    for c in range(n_cells):
        members = atoms[start[c]:start[c + 1]]
        assert np.all(np.diff(members) > 0)                              # ascending index
        assert np.all(cell[members] == c)
    # brute force on tiny input: cell_atoms equals a stable argsort of cell ids
    np.testing.assert_array_equal(atoms, np.argsort(cell, kind="stable"))


def test_bin_empty_cells_and_single_cell():
    cnt, start, atoms = O.bin_atoms(np.zeros(0, np.int32), 5)
    assert cnt.sum() == 0 and np.all(start == 0)
    cnt, start, atoms = O.bin_atoms(np.full(7, 3, np.int32), 5)
    np.testing.assert_array_equal(cnt, [0, 0, 0, 7, 0])
    np.testing.assert_array_equal(atoms, np.arange(7))


def test_wrap():
    L = np.array([10.0, 33.3, 44.376])
    rng = np.random.default_rng(7)
    inside = rng.random((3, 1000)) * L[:, None]
    np.testing.assert_array_equal(O.wrap(inside, L), inside)            # identity inside
    for k in (-3, -1, 1, 2):
        shifted = inside + k * L[:, None]
        w = O.wrap(shifted, L)
        assert np.all(w >= 0) and np.all(w < L[:, None])
        err = np.abs(w - inside)
        err = np.minimum(err, L[:, None] - err)                          # 0 and L are the same point
        assert err.max() <= 8 * np.finfo(float).eps * L.max() * (abs(k) + 1)
    edge = np.array([[-0.0, -1e-300, 10.0, np.nextafter(10.0, 0), -10.0]] * 3)
    w = O.wrap(edge, np.array([10.0, 10.0, 10.0]))
    assert np.all(w >= 0) and np.all(w < 10.0)
