"""Pins of the oracle's chain topology against the paper's printed example (Section 3.3)."""
import numpy as np

import oracle as O
from conftest import golden


def _per_atom_lists(terms, n_atoms):
    """Per-atom CSR in the layout of the paper's t_angles / t_bonds: for each atom, the
    terms containing it in ascending term ordinal, its position in the term (1-based) and
    the other atoms of the term in the term's own order."""
    index, ordinal, pos, others = [0], [], [], []
    for a in range(n_atoms):
        for t, term in enumerate(terms):
            term = list(term)
            if a in term:
                ordinal.append(t)
                pos.append(term.index(a) + 1)
                others.append([x for x in term if x != a])
        index.append(len(ordinal))
    return np.array(index), np.array(ordinal), np.array(pos), np.array(others)


def test_fig5_angle_lists():
    g = golden("fig5_t_angles.txt")
    terms = O.chain_terms(7, 3)
    index, ordinal, pos, others = _per_atom_lists(terms, 7)
    np.testing.assert_array_equal(index, g["index"])
    np.testing.assert_array_equal(ordinal, g["ang_idx"])
    np.testing.assert_array_equal(pos, g["pos"])
    np.testing.assert_array_equal(others[:, 0] + 1, g["at1"])
    np.testing.assert_array_equal(others[:, 1] + 1, g["at2"])


def test_fig4_bond_lists():
    g = golden("fig4_t_bonds.txt")
    terms = O.chain_terms(7, 2)
    index, _, _, others = _per_atom_lists(terms, 7)
    partners = others[:, 0] + 1
    np.testing.assert_array_equal(index[:2], g["printed_index_prefix"])
    np.testing.assert_array_equal(partners[:3], g["printed_bond_prefix"])
    # the rest follows from the same rule for a linear chain
    np.testing.assert_array_equal(index, [0, 1, 3, 5, 7, 9, 11, 12])
    np.testing.assert_array_equal(partners, [2, 1, 3, 2, 4, 3, 5, 4, 6, 5, 7, 6])


def test_term_multiplicities():
    """A per-atom gather does each bond twice, angle three times, dihedral four times
    (Sections 3.3): per-atom counts 1,2,..,2,1 / 1,2,3,..,3,2,1 / 1,2,3,4,..,4,3,2,1."""
    n = 300
    for k, n_terms in ((2, 299), (3, 298), (4, 297)):
        terms = O.chain_terms(n, k)
        assert len(terms) == n_terms
        counts = np.bincount(terms.ravel(), minlength=n)
        expect = np.minimum(np.minimum(np.arange(n) + 1, n - np.arange(n)), k)
        np.testing.assert_array_equal(counts, expect)
        assert counts.sum() == k * n_terms
