"""Neighbour-list mode (the paper's Verlet list, rebuilt when an atom has moved more than half
the skin, or every few steps) against the FP64 oracle and against the cell path, through the
C ABI."""
import numpy as np
import pytest

import oracle as O
from pe_melt import make_melt

pytestmark = pytest.mark.gpu

TOL = {"mixed": 1e-5, "fp64": 1e-10}
SKIN = 1.0


def norm_err(f, ref):
    frms = np.sqrt(np.mean(np.sum(ref ** 2, axis=0)))
    return float(np.max(np.sqrt(np.sum((f - ref) ** 2, axis=0))) / frms)


@pytest.fixture(scope="module")
def melt():
    return make_melt(10, density=0.80, T=500.0, seed_melt=1000, seed_vel=1001, jitter=0.05)


KERNELS = [4, 5]   # MD_LJ_NLIST (a list per atom), MD_LJ_NLIST_TILE (a list per cell)


def system(m, ff, precision, R=1, T0=0.0, skin=SKIN, every=10, kernel=4, **kw):
    from paper_1001_3764_amd.md import MDSystem
    print("nlist system: N=%d %s R=%d kernel=%d skin=%g every=%d %s" % (m.n_atoms, precision, R, kernel, skin,
                                                                      every, kw), flush=True)
    return MDSystem(ff, [m.n_chains], m.box[None, :], [T0], m.pos, m.vel, m.types, chain_len=m.chain_len,
                    precision=precision, cell_div=R, nl_skin=skin, nl_every=every, lj_kernel=kernel, **kw)


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("R", [1, 2])
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_nlist_bins_forces_energies(ff, melt, precision, R, kernel):
    """Bins are bit-exact on the grid of edge >= (rc + skin) / R; forces and energies from
    the list equal the oracle's."""
    s = system(melt, ff, precision, R, kernel=kernel)
    assert s.tuning() == (R, kernel)
    M, _, _ = s.grid(0)
    assert np.all(M == np.floor(melt.box * R / (ff["rc"] + SKIN)))
    start, atoms = s.bins()
    _, ostart, oatoms = O.bin_atoms(O.cell_index(melt.pos, melt.box, M), int(np.prod(M)))
    np.testing.assert_array_equal(start, ostart)
    np.testing.assert_array_equal(atoms, oatoms)
    f = s.forces()
    flj = s.forces(lj_only=True)
    e = s.energies()[0]
    fo_lj, eo = O.lj_cells(ff, melt.pos, melt.types, melt.box, 300)
    fo_b, eb = O.bonded(ff, melt.pos, melt.box, 300)
    print("nlist force error %s R=%d: LJ %.3e total %.3e" % (precision, R, norm_err(flj, fo_lj),
                                                              norm_err(f, fo_lj + fo_b)))
    assert norm_err(flj, fo_lj) <= TOL[precision] and norm_err(f, fo_lj + fo_b) <= TOL[precision]
    etol = 1e-12 if precision == "fp64" else 2e-6
    assert e["e_lj"] == pytest.approx(eo["e_lj"], rel=etol)
    assert e["e_lj_shifted"] == pytest.approx(eo["e_lj_shifted"], rel=etol)
    assert e["virial"] == pytest.approx(eo["virial_lj"] + eb["virial_bonded"], rel=max(etol, 1e-11))
    s.close()


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("precision,xtol", [("fp64", 1e-9), ("mixed", 1e-4)])
def test_nlist_trajectory_100_steps(ff, melt, precision, xtol, kernel):
    """100 NVE steps with the list rebuilt every 10: positions against the oracle (which
    searches the cells every step), checked every 25 steps, between builds too."""
    s = system(melt, ff, precision, 2, kernel=kernel)
    f0, _ = O.forces(ff, melt.pos, melt.types, melt.box, 300)
    p_o, v_o, f_o = melt.pos, melt.vel, f0
    worst = []
    for chunk in range(4):
        s.step(25)
        p_o, v_o, f_o, e_o = O.run(ff, p_o, v_o, f_o, melt.types, melt.box, 300, 25)
        p, v = s.state()
        d = p - p_o
        d -= melt.box[:, None] * np.round(d / melt.box[:, None])
        worst.append(float(np.abs(d).max()))
    e = s.energies()[0]
    print("nlist trajectory %s max|dx| per 25 steps: %s" % (precision, worst))
    assert worst[-1] <= xtol
    etol = 1e-9 if precision == "fp64" else 1e-4
    assert e["e_kin"] == pytest.approx(e_o["e_kin"], rel=etol)
    assert e["e_lj"] == pytest.approx(e_o["e_lj"], rel=etol * 10)
    s.close()


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_nlist_matches_cell_path(ff, melt, precision, kernel):
    """The same 30 Berendsen steps through the cell path and the list path (rebuilt every
    7): the same pairs, so the same trajectory up to summation order."""
    from paper_1001_3764_amd.md import MDSystem
    a = MDSystem(ff, [melt.n_chains], melt.box[None, :], [350.0], melt.pos, melt.vel, melt.types,
                 precision=precision, cell_div=2, lj_kernel=2)
    b = system(melt, ff, precision, 2, T0=350.0, every=7, kernel=kernel)
    a.step(30)
    b.step(30)
    pa, va = a.state()
    pb, vb = b.state()
    d = pa - pb
    d -= melt.box[:, None] * np.round(d / melt.box[:, None])
    print("cell vs list after 30 steps (%s): max|dx| %.3e" % (precision, np.abs(d).max()))
    assert np.abs(d).max() <= (1e-10 if precision == "fp64" else 1e-5)
    assert a.energies()[0]["temperature"] == pytest.approx(b.energies()[0]["temperature"],
                                                           rel=1e-12 if precision == "fp64" else 1e-6)
    a.close()
    b.close()


@pytest.mark.parametrize("kernel", KERNELS)
def test_nlist_graph_replay_and_timed_steps_are_bit_identical(ff, melt, kernel):
    a = system(melt, ff, "mixed", 2, T0=400.0, use_graph=False, every=4, kernel=kernel)
    b = system(melt, ff, "mixed", 2, T0=400.0, use_graph=True, every=4, kernel=kernel)
    c = system(melt, ff, "mixed", 2, T0=400.0, use_graph=False, every=4, kernel=kernel)
    for n in (3, 7, 6):
        a.step(n)
        b.step(n)
        ms = c.step_timed(n)
        assert ms["nlist_build"] >= 0
        pa, va = a.state()
        pb, vb = b.state()
        pc, vc = c.state()
        assert np.array_equal(pa, pb) and np.array_equal(va, vb)
        assert np.array_equal(pa, pc) and np.array_equal(va, vc)
    assert a.energies()[0] == b.energies()[0]
    for s in (a, b, c):
        s.close()


@pytest.mark.parametrize("kernel", KERNELS)
def test_nlist_batched_boxes(ff, kernel):
    """Three boxes of different sizes in one list-mode context: each box against the
    oracle after 20 steps (lists rebuilt every 6)."""
    from paper_1001_3764_amd.md import MDSystem
    melts = [make_melt(c, density=0.80, T=300.0 + 50 * k, seed_melt=900 + k, seed_vel=950 + k, jitter=0.05)
             for k, c in enumerate((4, 11, 7))]
    pos = np.concatenate([m.pos for m in melts], axis=1)
    vel = np.concatenate([m.vel for m in melts], axis=1)
    types = np.concatenate([m.types for m in melts])
    T0 = [280.0, 0.0, 420.0]
    s = MDSystem(ff, [m.n_chains for m in melts], np.stack([m.box for m in melts]), T0, pos, vel, types,
                 precision="mixed", cell_div=2, nl_skin=SKIN, nl_every=6, lj_kernel=kernel)
    f_all = s.forces()
    s.step(20)
    p_all, _ = s.state()
    off = 0
    for b, m in enumerate(melts):
        n = m.n_atoms
        fo, _ = O.forces(ff, m.pos, m.types, m.box, 300)
        assert norm_err(f_all[:, off:off + n], fo) <= TOL["mixed"]
        po, _, _, _ = O.run(ff, m.pos, m.vel, fo, m.types, m.box, 300, 20, T0=T0[b])
        d = p_all[:, off:off + n] - po
        d -= m.box[:, None] * np.round(d / m.box[:, None])
        print("box %d: max|dx| after 20 steps %.3e" % (b, np.abs(d).max()))
        assert np.abs(d).max() <= 1e-5
        off += n
    s.close()


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("precision,xtol", [("fp64", 1e-9), ("mixed", 1e-4)])
def test_nlist_rebuilds_on_displacement(ff, melt, kernel, precision, xtol):
    """Lists rebuilt only when an atom has moved more than half the skin (nl_every = 0), from the
    500 K melt: 100 steps against the oracle's, which searches the cells every step, and the
    graph-replayed and plain launch sequences bit-identical.  A 0.3 A skin makes the rebuilds
    frequent but not every step."""
    a = system(melt, ff, precision, 2, skin=0.3, every=0, kernel=kernel)
    b = system(melt, ff, precision, 2, skin=0.3, every=0, kernel=kernel, use_graph=True)
    f0, _ = O.forces(ff, melt.pos, melt.types, melt.box, 300)
    a.step(100)
    b.step(100)
    pa, va = a.state()
    pb, vb = b.state()
    assert np.array_equal(pa, pb) and np.array_equal(va, vb)
    a.energies()   # no device error
    builds = a.list_builds()
    assert b.list_builds() == builds
    po, _, _, _ = O.run(ff, melt.pos, melt.vel, f0, melt.types, melt.box, 300, 100)
    d = pa - po
    d -= melt.box[:, None] * np.round(d / melt.box[:, None])
    print("%s kernel %d: %d rebuilds in 100 steps, max|dx| %.3e A" % (precision, kernel, builds, np.abs(d).max()))
    assert 3 <= builds < 100
    assert np.abs(d).max() <= xtol
    a.close()
    b.close()


@pytest.mark.parametrize("kernel", KERNELS)
def test_nlist_thin_skin_rebuilds_every_step_it_must(ff, melt, kernel):
    """A skin far too thin for a fixed interval (0.02 A, nl_every = 100): the displacement check
    rebuilds whenever an atom has crossed half of it, so the run follows the cell path (the same
    pairs; only FP32 summation orders differ) and reports no error."""
    s = system(melt, ff, "mixed", 2, skin=0.02, every=100, kernel=kernel)
    from paper_1001_3764_amd.md import MDSystem
    c = MDSystem(ff, [melt.n_chains], melt.box[None, :], [0.0], melt.pos, melt.vel, melt.types,
                 chain_len=melt.chain_len, precision="mixed", cell_div=2, lj_kernel=2)
    s.step(60)
    c.step(60)
    s.energies()
    ps, _ = s.state()
    pc, _ = c.state()
    d = ps - pc
    d -= melt.box[:, None] * np.round(d / melt.box[:, None])
    builds = s.list_builds()
    print("kernel %d: %d rebuilds in 60 steps, max|dx| vs cell path %.3e A" % (kernel, builds, np.abs(d).max()))
    assert builds >= 30
    assert np.abs(d).max() <= 1e-4
    s.close()
    c.close()


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_nlist_full_lists_fall_back_to_the_stencil(ff, melt, kernel, precision):
    """The melt squeezed towards its box centre (positions scaled by 0.7 there): about 2.9 times
    the mean density, so atoms and cells in the dense region have more list partners than the
    capacity sized for the mean density holds.  Those walk their stencil instead; every force
    still equals the oracle's."""
    import dataclasses
    L = melt.box[:, None]
    p = L / 2 + 0.7 * (melt.pos - L / 2)
    m = dataclasses.replace(melt, pos=p)
    from scipy.spatial import cKDTree
    rl = ff["rc"] + SKIN
    counts = cKDTree(p.T, boxsize=melt.box).query_ball_point(p.T, rl, return_length=True)
    mean = 4.0 / 3.0 * np.pi * rl ** 3 * melt.n_atoms / np.prod(melt.box)
    assert counts.max() > 1.5 * mean + 64   # above the per-atom capacity for the mean density
    s = system(m, ff, precision, 2, kernel=kernel)
    flj = s.forces(lj_only=True)
    fo_lj, eo = O.lj_cells(ff, m.pos, m.types, m.box, 300)
    err = norm_err(flj, fo_lj)
    print("squeezed melt %s kernel %d: LJ error %.3e (densest atom %d partners, mean %.0f)"
          % (precision, kernel, err, counts.max(), mean))
    assert err <= TOL[precision]
    assert s.energies()[0]["e_lj"] == pytest.approx(eo["e_lj"], rel=1e-12 if precision == "fp64" else 2e-6)
    s.close()


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_nlist_pairs_at_the_cutoff(ff, precision, kernel):
    """Facing pairs at rc (1 + delta), delta in [-4e-7, 4e-7]: the list path counts exactly
    the FP64 pair set too."""
    rc = ff["rc"]
    deltas = np.array([-4e-7, -2e-7, -5e-8, -1e-8, 1e-8, 5e-8, 2e-7, 4e-7])
    n = deltas.size
    x = 5.0 + 1.53 * np.arange(n)
    pos = np.zeros((3, 2 * n))
    pos[0] = np.concatenate([x, x])
    pos[1] = np.concatenate([np.full(n, 5.0), 5.0 + rc * (1.0 + deltas)])
    pos[2] = 5.0
    box = np.array([40.0, 40.0, 40.0])
    types = np.zeros(2 * n, dtype=np.uint8)
    fo, _ = O.lj_brute(ff, pos, types, box, n)
    from paper_1001_3764_amd.md import MDSystem
    s = MDSystem(ff, [2], box[None, :], [0.0], pos, np.zeros_like(pos), types, chain_len=n,
                 precision=precision, cell_div=2, nl_skin=SKIN, nl_every=5, lj_kernel=kernel)
    flj = s.forces(lj_only=True)
    s.close()
    s6 = ff["sigma"][0] ** 6
    f_rc = 4 * ff["epsilon"][0] * (12 * s6 * s6 / rc ** 13 - 6 * s6 / rc ** 7)
    assert np.max(np.abs(flj - fo)) < 0.02 * abs(f_rc)


def test_nlist_autotuner_picks_a_list_kernel(ff, melt):
    """lj_kernel = 0 in list mode: the autotuner times both list layouts and the result
    still equals the oracle."""
    s = system(melt, ff, "mixed", 0, kernel=0)
    R, kern = s.tuning()
    print("list mode tuned to R=%d kernel=%d" % (R, kern), flush=True)
    assert R in (1, 2) and kern in KERNELS
    fo, _ = O.lj_cells(ff, melt.pos, melt.types, melt.box, 300)
    assert norm_err(s.forces(lj_only=True), fo) <= TOL["mixed"]
    s.close()
