"""Section 5 observables on the GPU (md_observables) against the oracle: exact pair-distance
and dihedral counts, chain shape to rounding."""
import numpy as np
import pytest

import oracle as O
from pe_melt import WORKLOADS, build_melts, make_melt

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def melt():
    return make_melt(10, density=0.80, T=500.0, seed_melt=1000, seed_vel=1001, jitter=0.05)


def system(ff, melts, **kw):
    from paper_1001_3764_amd.md import MDSystem
    pos = np.concatenate([m.pos for m in melts], axis=1)
    vel = np.concatenate([m.vel for m in melts], axis=1)
    types = np.concatenate([m.types for m in melts])
    print("observables system: %d boxes, N=%d %s" % (len(melts), pos.shape[1], kw), flush=True)
    return MDSystem(ff, [m.n_chains for m in melts], np.stack([m.box for m in melts]), [0.0] * len(melts), pos,
                    vel, types, chain_len=melts[0].chain_len, **kw)


def near_dihedral_edges(ff, pos, box, chain_len, n_bins, eps=1e-9):
    """Dihedrals whose oracle angle lies within eps of a histogram or class edge."""
    n = pos.shape[1]
    edges = np.concatenate([-np.pi + 2 * np.pi * np.arange(n_bins + 1) / max(n_bins, 1),
                            [-2 * np.pi / 3, 0.0, 2 * np.pi / 3]])
    hits = 0
    for p in range(n):
        if p % chain_len + 3 >= chain_len:
            continue
        s = [pos[:, p]]
        for a in range(1, 4):
            d = pos[:, p + a] - pos[:, p + a - 1]
            d -= box * np.round(d / box)
            s.append(s[-1] + d)
        _, _, phi = O.dihedral_term(ff, *s)
        hits += int(np.min(np.abs(edges - phi)) < eps)
    return hits


def check_box(ff, out, b, m, pos, rdf_bins, rmax, dih_bins, chain_off, check_edges=True):
    counts = O.pair_histogram(pos, m.box, m.chain_len, ff["excl_depth"], rmax, rdf_bins)
    np.testing.assert_array_equal(out["pair_counts"][b], counts)
    hist, cls = O.dihedral_stats(pos, m.box, m.chain_len, dih_bins)
    if check_edges:
        assert near_dihedral_edges(ff, pos, m.box, m.chain_len, dih_bins) == 0
    np.testing.assert_array_equal(out["dihedral_hist"][b], hist)
    np.testing.assert_array_equal(out["dihedral_classes"][b], cls)
    shape = O.chain_shape(ff, pos, m.types, m.box, m.chain_len)
    got = out["chain_shape"][chain_off:chain_off + m.n_chains]
    np.testing.assert_allclose(got[:, 0], shape[:, 0], rtol=1e-12)
    np.testing.assert_allclose(got[:, 1:], shape[:, 1:], rtol=0, atol=1e-10)
    return counts, cls


@pytest.mark.parametrize("R", [1, 2])
def test_observables_of_the_initial_melt(ff, melt, R):
    s = system(ff, [melt], precision="mixed", cell_div=R, lj_kernel=2)
    for rdf_bins, rmax, dih_bins in ((105, 10.5, 72), (700, 7.0, 0), (2048, 10.5, 2045)):
        out = s.observables(rdf_bins=rdf_bins, rdf_rmax=rmax, dih_bins=dih_bins)
        counts, cls = check_box(ff, out, 0, melt, melt.pos, rdf_bins, rmax, dih_bins, 0, check_edges=dih_bins < 100)
        print("R=%d bins=%d: %d pairs, trans/g+/g- %s" % (R, rdf_bins, counts.sum(), cls), flush=True)
    s.close()


@pytest.mark.parametrize("nl", [False, True])
def test_observables_after_steps(ff, melt, nl):
    """After 23 steps (between list builds in neighbour-list mode: the cell lists are those
    of the last build, the positions current)."""
    kw = dict(nl_skin=1.0, nl_every=10, lj_kernel=5) if nl else dict(lj_kernel=2)
    s = system(ff, [melt], precision="mixed", cell_div=2, use_graph=True, **kw)
    s.step(23)
    pos, _ = s.state()
    out = s.observables(rdf_bins=210, rdf_rmax=10.5, dih_bins=36)
    check_box(ff, out, 0, melt, pos, 210, 10.5, 36, 0)
    s.close()


def test_observables_of_batched_boxes(ff):
    melts = [make_melt(c, density=0.80, T=400.0, seed_melt=600 + c, seed_vel=650 + c, jitter=0.05)
             for c in (4, 9, 6)]
    s = system(ff, melts, precision="fp64", cell_div=1, lj_kernel=1)
    out = s.observables(rdf_bins=84, rdf_rmax=10.5, dih_bins=48)
    off = 0
    for b, m in enumerate(melts):
        check_box(ff, out, b, m, m.pos, 84, 10.5, 48, off)
        off += m.n_chains
    s.close()


def test_observables_at_full_size(ff):
    """The 300,000-atom melt in the bench's launch configuration (autotuned grid), 5 steps
    in: the grown melt places every dihedral at exactly 180 or +-60 deg, on histogram edges,
    where rounding alone picks the bin."""
    import os
    O.set_threads(max(1, min(16, os.cpu_count() or 1)))
    m = build_melts(WORKLOADS["melt300k_mixed"], max(1, min(16, os.cpu_count() or 1)))[0]
    s = system(ff, [m], precision="mixed", cell_div=0, lj_kernel=0, use_graph=True)
    s.step(5)
    pos, _ = s.state()
    out = s.observables(rdf_bins=210, rdf_rmax=10.5, dih_bins=72)
    counts, cls = check_box(ff, out, 0, m, pos, 210, 10.5, 72, 0, check_edges=False)
    print("300k: %d pairs, trans fraction %.4f" % (counts.sum(), cls[0] / cls.sum()), flush=True)
    s.close()


def test_observable_arguments_are_checked(ff, melt):
    from paper_1001_3764_amd.md import MD_ERR_ARG, MDError
    s = system(ff, [melt], precision="mixed", cell_div=1, lj_kernel=1)
    for kw in (dict(rdf_rmax=ff["rc"] * 1.01), dict(rdf_bins=0), dict(rdf_bins=2049), dict(dih_bins=2046)):
        with pytest.raises(MDError) as ex:
            s.observables(**kw)
        assert ex.value.status == MD_ERR_ARG
    s.close()


def test_end_to_end_acf_against_the_oracle(ff):
    """md_ree_acf against the oracle's ora_ree_acf: three boxes in one context, the reference at
    init, then after 40 and 100 steps; then a new reference, 30 steps on.  Both sums are over
    the same FP64 bond vectors in different orders, so they agree to rounding (1e-12)."""
    from paper_1001_3764_amd.md import MDSystem
    melts = [make_melt(c, density=0.80, T=450.0, seed_melt=700 + c, seed_vel=710 + c, jitter=0.05)
             for c in (4, 9, 6)]
    pos = np.concatenate([m.pos for m in melts], axis=1)
    vel = np.concatenate([m.vel for m in melts], axis=1)
    types = np.concatenate([m.types for m in melts])
    s = MDSystem(ff, [m.n_chains for m in melts], np.stack([m.box for m in melts]), [0.0, 300.0, 0.0], pos, vel,
                 types, precision="mixed", cell_div=2, lj_kernel=2, use_graph=True)
    assert np.allclose(s.ree_acf(), 1.0, rtol=0, atol=1e-15)
    ref = pos
    for n in (40, 60):
        s.step(n)
        p, _ = s.state()
        got = s.ree_acf()
        off = 0
        for b, m in enumerate(melts):
            sl = slice(off, off + m.n_atoms)
            want = O.ree_acf(ref[:, sl], p[:, sl], m.box, m.chain_len)
            print("box %d: acf %.15f (oracle %.15f)" % (b, got[b], want), flush=True)
            assert got[b] == pytest.approx(want, rel=0, abs=1e-12)
            off += m.n_atoms
    s.ree_reference()
    ref, _ = s.state()
    s.step(30)
    p, _ = s.state()
    got = s.ree_acf()
    off = 0
    for b, m in enumerate(melts):
        sl = slice(off, off + m.n_atoms)
        assert got[b] == pytest.approx(O.ree_acf(ref[:, sl], p[:, sl], m.box, m.chain_len), rel=0, abs=1e-12)
        off += m.n_atoms
    s.close()
