"""GPU parity against the FP64 oracle, through the C ABI (gfx950)."""
import numpy as np
import pytest

import oracle as O
from pe_melt import make_melt

pytestmark = pytest.mark.gpu

# Force error metric: max_i |F_gpu,i - F_ora,i| / F_rms(ora), F_rms = sqrt(mean_i |F_ora,i|^2)
TOL_MIXED = 1e-5     # FP32 forces
TOL_FP64 = 1e-10     # FP64 forces (summation order and cell-relative differences differ)


def norm_err(f, ref):
    frms = np.sqrt(np.mean(np.sum(ref ** 2, axis=0)))
    return float(np.max(np.sqrt(np.sum((f - ref) ** 2, axis=0))) / frms)


def make_system(m, ff, precision, R=1, T0=0.0, **kw):
    from paper_1001_3764_amd.md import MDSystem
    print("system: N=%d precision=%s R=%d T0=%g %s" % (m.n_atoms, precision, R, T0, kw), flush=True)
    return MDSystem(ff, [m.n_chains], m.box[None, :], [T0], m.pos, m.vel, m.types,
                    chain_len=m.chain_len, precision=precision, cell_div=R, **kw)


@pytest.fixture(scope="module")
def melt():
    return make_melt(10, density=0.80, T=500.0, seed_melt=1000, seed_vel=1001, jitter=0.05)


@pytest.mark.parametrize("R", [1, 2])
def test_bins_bit_exact(ff, melt, R):
    s = make_system(melt, ff, "mixed", R)
    start, atoms = s.bins()
    M, co, ao = s.grid(0)
    assert co == 0 and ao == 0
    assert np.all(M == np.floor(melt.box * R / ff["rc"]))
    cell = O.cell_index(melt.pos, melt.box, M)
    cnt, ostart, oatoms = O.bin_atoms(cell, int(np.prod(M)))
    np.testing.assert_array_equal(start, ostart)
    np.testing.assert_array_equal(atoms, oatoms)
    s.close()


@pytest.mark.parametrize("M", [40, 41])
def test_bins_bit_exact_at_the_scan_path_boundary(ff, melt, M):
    """40^3 = 64,000 cells fill 16 scan tiles of 4,096 (the one-launch scan, whose last block sums
    the counts of 15 tiles); 41^3 = 68,921 fill 17 (tile totals first, then the scan).  The
    melt's positions are stretched over the larger box so that every tile holds atoms."""
    import dataclasses
    R = 2
    box = np.full(3, (M + 0.5) * ff["rc"] / R)
    m = dataclasses.replace(melt, box=box, pos=melt.pos * (box / melt.box)[:, None])
    s = make_system(m, ff, "mixed", R)
    start, atoms = s.bins()
    Mg, _, _ = s.grid(0)
    assert np.all(Mg == M)
    cell = O.cell_index(m.pos, m.box, Mg)
    cnt, ostart, oatoms = O.bin_atoms(cell, int(np.prod(Mg)))
    assert np.count_nonzero(np.add.reduceat(cnt, np.arange(0, cnt.size, 4096))) == -(-cnt.size // 4096)
    np.testing.assert_array_equal(start, ostart)
    np.testing.assert_array_equal(atoms, oatoms)
    s.close()


def test_wrap_and_bins_bit_exact_from_outside_the_box(ff, melt):
    """Positions shifted by whole and fractional box lengths: the GPU wrap and cell index
    must equal the oracle's bit for bit."""
    rng = np.random.default_rng(12)
    p = melt.pos + melt.box[:, None] * rng.integers(-2, 3, size=melt.pos.shape)
    p[:, :50] += 1e-13          # a few just past the faces
    from paper_1001_3764_amd.md import MDSystem
    s = MDSystem(ff, [melt.n_chains], melt.box[None, :], [0.0], p, melt.vel, melt.types,
                 precision="fp64", cell_div=1)
    pos, _ = s.state()
    np.testing.assert_array_equal(pos, O.wrap(p, melt.box))
    start, atoms = s.bins()
    M, _, _ = s.grid(0)
    cnt, ostart, oatoms = O.bin_atoms(O.cell_index(O.wrap(p, melt.box), melt.box, M), int(np.prod(M)))
    np.testing.assert_array_equal(start, ostart)
    np.testing.assert_array_equal(atoms, oatoms)
    s.close()


@pytest.mark.parametrize("kernel", [1, 2, 3, 6])
@pytest.mark.parametrize("precision,tol", [("fp64", TOL_FP64), ("mixed", TOL_MIXED)])
@pytest.mark.parametrize("R", [1, 2])
def test_forces_and_energies(ff, melt, precision, tol, R, kernel):
    s = make_system(melt, ff, precision, R, lj_kernel=kernel)
    f = s.forces()
    flj = s.forces(lj_only=True)
    e = s.energies()[0]
    fo_lj, eo = O.lj_cells(ff, melt.pos, melt.types, melt.box, 300)
    fo_b, eb = O.bonded(ff, melt.pos, melt.box, 300)
    err_lj = norm_err(flj, fo_lj)
    err_b = norm_err(f - flj, fo_b)
    err = norm_err(f, fo_lj + fo_b)
    print("force error %s R=%d kernel=%d: LJ %.3e bonded %.3e total %.3e" % (precision, R, kernel, err_lj, err_b, err))
    assert err_lj <= tol and err_b <= tol and err <= tol
    # energies: compensated FP64 sums of per-pair/per-term values
    etol = 1e-12 if precision == "fp64" else 2e-6
    assert e["e_lj"] == pytest.approx(eo["e_lj"], rel=etol)
    assert e["e_lj_shifted"] == pytest.approx(eo["e_lj_shifted"], rel=etol)
    assert e["e_bond"] == pytest.approx(eb["e_bond"], rel=etol)
    assert e["e_angle"] == pytest.approx(eb["e_angle"], rel=etol)
    assert e["e_dih"] == pytest.approx(eb["e_dih"], rel=etol)
    assert e["virial"] == pytest.approx(eo["virial_lj"] + eb["virial_bonded"], rel=max(etol, 1e-11))
    ke, T = O.kinetic(ff, melt.vel, melt.types)
    assert e["e_kin"] == pytest.approx(ke, rel=1e-13)
    assert e["temperature"] == pytest.approx(T, rel=1e-13)
    # Newton's third law on the GPU forces
    assert np.abs(f.sum(axis=1)).max() <= (1e-9 if precision == "fp64" else 1e-4) * np.abs(f).sum() / f.shape[1]
    s.close()


@pytest.mark.parametrize("homes", [4, 8, 16])
@pytest.mark.parametrize("kernel,R,skin", [(2, 1, 0.0), (2, 2, 0.0), (3, 2, 0.0), (5, 2, 1.0)])
def test_tile_homes_per_wave(ff, melt, homes, kernel, R, skin):
    """The cell tile with 4, 8 or 16 home atoms per pass of a wavefront (the autotuner's
    atoms-per-wave choice): forces, energies and a 50-step trajectory against the oracle; the
    choice is reported back by md_tuning."""
    kw = dict(lj_kernel=kernel, tile_homes=homes)
    if skin:
        kw.update(nl_skin=skin, nl_every=0)
    s = make_system(melt, ff, "mixed", R, **kw)
    assert s.tuning(homes=True) == (R, kernel, homes)
    f = s.forces()
    e = s.energies()[0]
    fo, eo = O.forces(ff, melt.pos, melt.types, melt.box, 300)
    err = norm_err(f, fo)
    print("homes=%d kernel=%d R=%d: force error %.3e" % (homes, kernel, R, err), flush=True)
    assert err <= TOL_MIXED
    assert e["e_lj"] == pytest.approx(eo["e_lj"], rel=2e-6)
    s.step(50)
    p, _ = s.state()
    po, _, _, _ = O.run(ff, melt.pos, melt.vel, fo, melt.types, melt.box, 300, 50)
    d = p - po
    d -= melt.box[:, None] * np.round(d / melt.box[:, None])
    assert np.abs(d).max() <= 1e-4
    s.close()


def test_types_beyond_the_force_field_are_refused(ff, melt):
    """Table I has two united atoms (types 0 and 1): a type 2 fails the set-up with MD_ERR_ARG."""
    from paper_1001_3764_amd.md import MD_ERR_ARG, MDError
    t = melt.types.copy()
    t[1234] = 2
    from paper_1001_3764_amd.md import MDSystem
    with pytest.raises(MDError) as ex:
        MDSystem(ff, [melt.n_chains], melt.box[None, :], [0.0], melt.pos, melt.vel, t, precision="mixed", cell_div=1)
    assert ex.value.status == MD_ERR_ARG


def forced_contacts(melt, targets, seed=5):
    """A copy of the melt in which, for each target distance, one atom is moved towards a
    nearby atom of another chain until the two are that far apart (minimum image), keeping every
    other non-bonded distance of the moved atom above 2.8 A.  Returns the melt and the pairs."""
    import dataclasses
    from scipy.spatial import cKDTree
    p = melt.pos.copy()
    L = melt.box
    rng = np.random.default_rng(seed)
    pairs, used = [], set()
    for r in targets:
        for i in rng.permutation(melt.n_atoms):
            tree = cKDTree(np.mod(p, L[:, None]).T, boxsize=L)
            js = [j for j in tree.query_ball_point(np.mod(p[:, i], L), 5.0)
                  if j // melt.chain_len != i // melt.chain_len and j not in used and i not in used]
            if not js:
                continue
            j = js[0]
            d = p[:, j] - p[:, i]
            d -= L * np.round(d / L)
            xj = p[:, i] + d * (r / np.linalg.norm(d))
            near = tree.query_ball_point(np.mod(xj, L), 2.8)
            others = [k for k in near if k not in (i, j) and (k // melt.chain_len != j // melt.chain_len
                                                          or abs(k - j) > 3)]
            if others:
                continue
            p[:, j] = np.mod(xj, L)
            pairs.append((int(i), int(j), r))
            used.update((int(i), int(j)))
            break
    assert len(pairs) == len(targets)
    return dataclasses.replace(melt, pos=p), pairs


CONTACTS = [1.9, 2.05, 2.2, 2.45, 2.58, 2.65]   # either side of 0.75 sigma = 2.6025 A


@pytest.mark.parametrize("kernel,R,skin", [(1, 1, 0.0), (2, 1, 0.0), (2, 2, 0.0), (3, 2, 0.0), (6, 2, 0.0),
                                           (4, 2, 1.0), (5, 2, 1.0)])
def test_close_contacts_in_fp64(ff, melt, kernel, R, skin):
    """Forced close contacts (1.9-2.65 A, LJ forces up to ~30 times the melt's RMS force): the mixed
    form evaluates those below 0.75 sigma in FP64, so even there the error stays within 1e-5 of
    the RMS force of the other atoms (FP32 alone errs by a few 1e-7 of the contact force, i.e.
    several 1e-5 of it)."""
    m, pairs = forced_contacts(melt, CONTACTS)
    kw = dict(lj_kernel=kernel)
    if skin:
        kw.update(nl_skin=skin, nl_every=10)
    s = make_system(m, ff, "mixed", R, **kw)
    flj = s.forces(lj_only=True)
    f = s.forces()
    e = s.energies()[0]
    fo_lj, eo = O.lj_cells(ff, m.pos, m.types, m.box, 300)
    fo_b, eb = O.bonded(ff, m.pos, m.box, 300)
    fo = fo_lj + fo_b
    touched = np.array(sorted({a for i, j, _ in pairs for a in (i, j)}))
    rest = np.setdiff1d(np.arange(m.n_atoms), touched)
    frms_rest = np.sqrt(np.mean(np.sum(fo[:, rest] ** 2, axis=0)))
    d_lj = np.sqrt(np.sum((flj - fo_lj) ** 2, axis=0))
    print("contacts kernel=%d R=%d: |F| at contacts / F_rms(rest) up to %.1f; LJ error there %.3e, "
          "elsewhere %.3e (over F_rms of the rest)"
          % (kernel, R, np.sqrt(np.sum(fo[:, touched] ** 2, axis=0)).max() / frms_rest,
             d_lj[touched].max() / frms_rest, d_lj[rest].max() / frms_rest), flush=True)
    assert np.sqrt(np.sum(fo_lj[:, touched] ** 2, axis=0)).max() > 25 * frms_rest
    # FP32 would err by ~1e-5 at the 1.9 A contact and ~5e-6 at 2.05 A
    assert d_lj[touched].max() <= 3e-6 * frms_rest
    assert d_lj.max() <= 1e-5 * frms_rest
    assert norm_err(f, fo) <= TOL_MIXED
    assert e["e_lj"] == pytest.approx(eo["e_lj"], rel=2e-6)
    assert e["e_lj_shifted"] == pytest.approx(eo["e_lj_shifted"], rel=2e-6)
    assert e["virial"] == pytest.approx(eo["virial_lj"] + eb["virial_bonded"], rel=2e-6)
    s.close()


@pytest.mark.parametrize("kernel", [1, 2, 6])
@pytest.mark.parametrize("precision,xtol", [("fp64", 1e-9), ("mixed", 1e-4)])
def test_trajectory_100_steps(ff, melt, precision, xtol, kernel):
    """The 3,000-atom melt, NVE, 100 steps of 1 fs: positions against the oracle."""
    s = make_system(melt, ff, precision, 1, lj_kernel=kernel)
    f0, _ = O.forces(ff, melt.pos, melt.types, melt.box, 300)
    worst = []
    p_o, v_o, f_o = melt.pos, melt.vel, f0
    for chunk in range(4):
        s.step(25)
        p_o, v_o, f_o, e_o = O.run(ff, p_o, v_o, f_o, melt.types, melt.box, 300, 25)
        p, v = s.state()
        d = p - p_o
        d -= melt.box[:, None] * np.round(d / melt.box[:, None])
        worst.append(float(np.abs(d).max()))
    e = s.energies()[0]
    print("trajectory %s max|dx| per 25 steps: %s" % (precision, worst))
    assert worst[-1] <= xtol
    assert e["step"] == 100
    etol = 1e-9 if precision == "fp64" else 1e-4
    assert e["e_kin"] == pytest.approx(e_o["e_kin"], rel=etol)
    assert e["e_lj"] == pytest.approx(e_o["e_lj"], rel=etol * 10)
    s.close()


@pytest.mark.parametrize("precision,kernel,homes", [("fp64", 2, 0), ("mixed", 1, 0), ("mixed", 2, 4),
                                                    ("mixed", 2, 8), ("mixed", 2, 16)])
def test_short_chains(ff, precision, kernel, homes):
    """250 chains of 12 sites (3,000 atoms, a sixth of them CH3 ends): chain ends everywhere, so
    the exclusion windows are clipped at most homes' chain ends and many bonded terms are end
    terms.  Bins bit-exact, forces within the bar, and 40 Berendsen steps against the oracle."""
    m = make_melt(250, chain_len=12, density=0.80, T=500.0, seed_melt=2024, seed_vel=2025, jitter=0.05)
    s = make_system(m, ff, precision, 2, T0=350.0, lj_kernel=kernel, tile_homes=homes)
    start, atoms = s.bins()
    M, _, _ = s.grid(0)
    _, ostart, oatoms = O.bin_atoms(O.cell_index(m.pos, m.box, M), int(np.prod(M)))
    assert np.array_equal(start, ostart) and np.array_equal(atoms, oatoms)
    fo, _ = O.forces(ff, m.pos, m.types, m.box, 12)
    err = norm_err(s.forces(), fo)
    print("short chains %s kernel %d homes %d: force error %.3e" % (precision, kernel, homes, err))
    assert err <= (TOL_FP64 if precision == "fp64" else TOL_MIXED)
    s.step(40)
    p_o, v_o, f_o, e_o = O.run(ff, m.pos, m.vel, fo, m.types, m.box, 12, 40, T0=350.0)
    p, v = s.state()
    d = p - p_o
    d -= m.box[:, None] * np.round(d / m.box[:, None])
    assert np.abs(d).max() <= (1e-9 if precision == "fp64" else 1e-4)
    e = s.energies()[0]
    assert e["temperature"] == pytest.approx(e_o["temperature"], rel=1e-9 if precision == "fp64" else 1e-4)
    s.close()


@pytest.mark.parametrize("precision,kernel", [("fp64", 1), ("fp64", 2), ("mixed", 1), ("mixed", 2), ("mixed", 6)])
def test_orthorhombic_box(ff, melt, precision, kernel):
    """The 3,000-atom melt stretched to an orthorhombic box of the same volume (x 1.15, y 0.95,
    z 1 / 1.0925): a different cell count along each axis, so the wrap, the cell coordinates,
    the stencil shifts and the sentinel are exercised per axis.  Bins bit-exact, forces within
    the bar, and 30 NVE steps against the oracle."""
    from paper_1001_3764_amd.md import MDSystem
    scale = np.array([1.15, 0.95, 1.0 / (1.15 * 0.95)])
    box = melt.box * scale
    pos = np.ascontiguousarray(np.mod(melt.pos * scale[:, None], box[:, None]))
    s = MDSystem(ff, [melt.n_chains], box[None, :], [0.0], pos, melt.vel, melt.types, chain_len=300,
                 precision=precision, cell_div=2, lj_kernel=kernel)
    start, atoms = s.bins()
    M, _, _ = s.grid(0)
    assert len(set(int(x) for x in M)) == 3
    _, ostart, oatoms = O.bin_atoms(O.cell_index(pos, box, M), int(np.prod(M)))
    assert np.array_equal(start, ostart) and np.array_equal(atoms, oatoms)
    fo, _ = O.forces(ff, pos, melt.types, box, 300)
    err = norm_err(s.forces(), fo)
    print("orthorhombic %s kernel %d (M = %s): force error %.3e" % (precision, kernel, [int(x) for x in M], err))
    assert err <= (TOL_FP64 if precision == "fp64" else TOL_MIXED)
    s.step(30)
    p_o, _, _, _ = O.run(ff, pos, melt.vel, fo, melt.types, box, 300, 30)
    p, _ = s.state()
    d = p - p_o
    d -= box[:, None] * np.round(d / box[:, None])
    assert np.abs(d).max() <= (1e-9 if precision == "fp64" else 1e-4)
    s.close()


@pytest.mark.parametrize("n_chains,R", [(56, 2), (90, 1)])
@pytest.mark.parametrize("precision,kernel", [("fp64", 2), ("mixed", 1), ("mixed", 2), ("mixed", 6)])
def test_smallest_boxes(ff, n_chains, R, precision, kernel):
    """Boxes with the fewest cells the stencil allows, 2R + 1 per axis (5 at R = 2 in a 27.1 A box,
    3 at R = 1 in a 31.7 A box; chains of 12 sites): every neighbour cell is reached through the
    periodic wrap from some home.  Bins bit-exact, forces within the bar, 20 steps against the
    oracle."""
    from paper_1001_3764_amd.md import MDSystem
    m = make_melt(n_chains, chain_len=12, density=0.80, T=500.0, seed_melt=77, seed_vel=78, jitter=0.05)
    s = MDSystem(ff, [m.n_chains], m.box[None, :], [0.0], m.pos, m.vel, m.types, chain_len=12,
                 precision=precision, cell_div=R, lj_kernel=kernel)
    start, atoms = s.bins()
    M, _, _ = s.grid(0)
    assert [int(x) for x in M] == [2 * R + 1] * 3
    _, ostart, oatoms = O.bin_atoms(O.cell_index(m.pos, m.box, M), int(np.prod(M)))
    assert np.array_equal(start, ostart) and np.array_equal(atoms, oatoms)
    # the oracle's grid search on the same stencil (a 27-cell grid of edge >= rc needs 3 rc), and
    # its LJ part against the brute-force pair sum
    fo, _ = O.forces(ff, m.pos, m.types, m.box, 12, R=R)
    fb, _ = O.lj_brute(ff, m.pos, m.types, m.box, 12)
    fl, _ = O.lj_cells(ff, m.pos, m.types, m.box, 12, R=R)
    assert norm_err(fl, fb) <= 1e-12
    err = norm_err(s.forces(), fo)
    print("smallest box R=%d %s kernel %d: force error %.3e" % (R, precision, kernel, err))
    assert err <= (TOL_FP64 if precision == "fp64" else TOL_MIXED)
    s.step(20)
    p_o, _, _, _ = O.run(ff, m.pos, m.vel, fo, m.types, m.box, 12, 20, R=R)
    p, _ = s.state()
    d = p - p_o
    d -= m.box[:, None] * np.round(d / m.box[:, None])
    assert np.abs(d).max() <= (1e-9 if precision == "fp64" else 1e-4)
    s.close()


@pytest.mark.parametrize("precision,kernel", [("fp64", 2), ("mixed", 1), ("mixed", 2), ("mixed", 6)])
def test_sparse_box(ff, precision, kernel):
    """Six 300-site chains at 0.05 g/cm^3 (1,800 atoms in a 94 A box): most cells empty, most
    stencils nearly so, so the empty-cell, empty-group and short-list paths all run.  Bins
    bit-exact, forces within the bar, 30 steps against the oracle."""
    from paper_1001_3764_amd.md import MDSystem
    m = make_melt(6, chain_len=300, density=0.05, T=500.0, seed_melt=91, seed_vel=92, jitter=0.05)
    s = MDSystem(ff, [m.n_chains], m.box[None, :], [0.0], m.pos, m.vel, m.types, chain_len=300,
                 precision=precision, cell_div=2, lj_kernel=kernel)
    start, atoms = s.bins()
    M, _, _ = s.grid(0)
    counts = np.diff(start)
    assert (counts == 0).mean() > 0.5
    _, ostart, oatoms = O.bin_atoms(O.cell_index(m.pos, m.box, M), int(np.prod(M)))
    assert np.array_equal(start, ostart) and np.array_equal(atoms, oatoms)
    fo, _ = O.forces(ff, m.pos, m.types, m.box, 300)
    err = norm_err(s.forces(), fo)
    print("sparse box %s kernel %d: %.0f%% empty cells, force error %.3e"
          % (precision, kernel, 100 * (counts == 0).mean(), err))
    assert err <= (TOL_FP64 if precision == "fp64" else TOL_MIXED)
    s.step(30)
    p_o, _, _, _ = O.run(ff, m.pos, m.vel, fo, m.types, m.box, 300, 30)
    p, _ = s.state()
    d = p - p_o
    d -= m.box[:, None] * np.round(d / m.box[:, None])
    assert np.abs(d).max() <= (1e-9 if precision == "fp64" else 1e-4)
    s.close()


@pytest.mark.parametrize("R", [1, 2])
@pytest.mark.parametrize("precision,kernel", [("fp64", 2), ("mixed", 1), ("mixed", 2), ("mixed", 6)])
def test_compressed_melt(ff, melt, R, precision, kernel):
    """The 3,000-atom melt squeezed to 0.8 of its box edge (1.95 times the density): stencils
    longer than one list chunk at R = 2 (walked unfiltered, chunk by chunk), and thousands of
    pairs closer than 0.75 sigma, so groups exceed the close-contact queue and take the full
    walk.  Forces within the bar, and 5 steps against the oracle."""
    from paper_1001_3764_amd.md import MDSystem
    box = melt.box * 0.8
    pos = np.ascontiguousarray(melt.pos * 0.8)
    s = MDSystem(ff, [melt.n_chains], box[None, :], [0.0], pos, melt.vel, melt.types, chain_len=300,
                 precision=precision, cell_div=R, lj_kernel=kernel)
    fo, _ = O.forces(ff, pos, melt.types, box, 300)
    err = norm_err(s.forces(), fo)
    print("compressed R=%d %s kernel %d: force error %.3e" % (R, precision, kernel, err))
    assert err <= (TOL_FP64 if precision == "fp64" else TOL_MIXED)
    s.step(5)
    p_o, _, _, _ = O.run(ff, pos, melt.vel, fo, melt.types, box, 300, 5)
    p, _ = s.state()
    d = p - p_o
    d -= box[:, None] * np.round(d / box[:, None])
    assert np.abs(d).max() <= (1e-9 if precision == "fp64" else 1e-4)
    s.close()


def test_berendsen_quench_matches_oracle(ff, melt):
    s = make_system(melt, ff, "fp64", 1, T0=300.0)
    f0, _ = O.forces(ff, melt.pos, melt.types, melt.box, 300)
    s.step(20)
    p_o, v_o, f_o, e_o = O.run(ff, melt.pos, melt.vel, f0, melt.types, melt.box, 300, 20, T0=300.0)
    e = s.energies()[0]
    assert e["temperature"] == pytest.approx(e_o["temperature"], rel=1e-10)
    p, v = s.state()
    assert np.abs(v - v_o).max() < 1e-10
    s.close()


def test_graph_replay_is_bit_identical(ff, melt):
    a = make_system(melt, ff, "mixed", 1, T0=400.0, use_graph=False)
    b = make_system(melt, ff, "mixed", 1, T0=400.0, use_graph=True)
    for _ in range(3):
        a.step(7)
        b.step(7)
        pa, va = a.state()
        pb, vb = b.state()
        assert np.array_equal(pa, pb) and np.array_equal(va, vb)
    assert a.energies()[0] == b.energies()[0]
    a.close()
    b.close()


@pytest.mark.parametrize("precision,com,graph", [("mixed", False, False), ("mixed", True, True),
                                                  ("fp64", False, True), ("fp64", True, False)])
def test_timed_step_matches_plain_step(ff, melt, precision, com, graph):
    """Plain steps (graph-replayed or not) and timed steps (an event around each phase) must give
    the same bits, with and without the COM removal, at T0 > 0."""
    a = make_system(melt, ff, precision, 1, T0=350.0, remove_com=com, use_graph=graph)
    b = make_system(melt, ff, precision, 1, T0=350.0, remove_com=com, use_graph=False)
    for n in (5, 3):
        a.step(n)
        ms = b.step_timed(n)
        assert set(ms) >= {"lj", "bonded_kick", "integrate_bin"} and all(v >= 0 for v in ms.values())
        pa, va = a.state()
        pb, vb = b.state()
        assert np.array_equal(pa, pb) and np.array_equal(va, vb)
    assert a.energies()[0] == b.energies()[0]
    a.close()
    b.close()


def test_general_types_and_dihedral_phase(ff, melt):
    """Unequal LJ types (Lorentz-Berthelot mixing) and a dihedral with n = 2, phi_s = 30 deg:
    the general code paths of both kernels against the oracle."""
    ffg = dict(ff, sigma=(3.47, 3.70), epsilon=(0.0951, 0.1200), n_dih=2, phis_deg=30.0)
    fo_lj, eo = O.lj_cells(ffg, melt.pos, melt.types, melt.box, 300)
    fo_b, eb = O.bonded(ffg, melt.pos, melt.box, 300)
    for precision, tol in (("fp64", TOL_FP64), ("mixed", TOL_MIXED)):
        for kernel in (1, 2, 6):
            s = make_system(melt, ffg, precision, 1, lj_kernel=kernel)
            f = s.forces()
            flj = s.forces(lj_only=True)
            e = s.energies()[0]
            assert norm_err(flj, fo_lj) <= tol
            assert norm_err(f - flj, fo_b) <= tol
            assert e["e_dih"] == pytest.approx(eb["e_dih"], rel=1e-12 if precision == "fp64" else 2e-6)
            s.close()


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("R,kernel", [(1, 1), (1, 2), (2, 2), (2, 3), (1, 6), (2, 6)])
def test_pairs_at_the_cutoff(ff, precision, R, kernel):
    """Two straight 8-atom chains side by side, atom k of one facing atom k of the other at
    r = rc (1 + delta_k), delta_k from -4e-7 to +4e-7: inside the FP32 uncertainty of r^2.
    The LJ pair set must be the FP64 one: each facing pair adds |F(rc)| ~ 3e-4 kcal/mol/A
    or nothing, so every atom's LJ force is compared with the oracle far below that."""
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
    # the oracle's own decision: the facing pair counts iff delta < 0
    d = pos[:, n:] - pos[:, :n]
    inside = np.sum(d * d, axis=0) < rc * rc
    assert np.array_equal(inside, deltas < 0)
    from paper_1001_3764_amd.md import MDSystem
    print("cutoff pairs: precision=%s R=%d kernel=%d" % (precision, R, kernel), flush=True)
    s = MDSystem(ff, [2], box[None, :], [0.0], pos, np.zeros_like(pos), types, chain_len=n,
                 precision=precision, cell_div=R, lj_kernel=kernel)
    flj = s.forces(lj_only=True)
    s.close()
    s6 = ff["sigma"][0] ** 6
    f_rc = 4 * ff["epsilon"][0] * (12 * s6 * s6 / rc ** 13 - 6 * s6 / rc ** 7)
    assert np.max(np.abs(flj - fo)) < 0.02 * abs(f_rc)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("R,kernel,nl", [(1, 2, False), (2, 2, False), (2, 3, False), (2, 1, False), (1, 4, True),
                                         (1, 5, True), (2, 5, True), (1, 6, False), (2, 6, False)])
def test_many_pairs_at_the_cutoff(ff, precision, R, kernel, nl):
    """One atom with 100 partners on a sphere of radius rc (1 + delta), |delta| <= 4e-7: more
    band pairs than the cell tile's queue holds (64), spread over more than its 8 recorded
    steps, so the group falls back to walking all of its candidates again.  The pair set must
    still be the FP64 one."""
    rc = ff["rc"]
    rng = np.random.default_rng(12)
    m = 100
    g = (1 + 5 ** 0.5) / 2
    t = np.arange(m) + 0.5
    u = np.stack([np.cos(2 * np.pi * t / g) * np.sqrt(1 - (1 - 2 * t / m) ** 2),
                  np.sin(2 * np.pi * t / g) * np.sqrt(1 - (1 - 2 * t / m) ** 2), 1 - 2 * t / m])
    delta = rng.uniform(1e-9, 4e-7, m) * np.where(np.arange(m) % 2 == 0, 1.0, -1.0)
    centre = np.array([20.0, 20.0, 20.0])
    sphere = centre[:, None] + rc * (1 + delta) * u
    # chains of 4: the centre and three atoms far from everything; then the sphere, 4 at a time
    far = np.array([[3.0, 3.0, 3.0], [3.0, 7.0, 3.0], [7.0, 3.0, 3.0]]).T
    pos = np.concatenate([centre[:, None], far, sphere], axis=1)
    box = np.array([40.0, 40.0, 40.0])
    types = np.zeros(pos.shape[1], dtype=np.uint8)
    fo, _ = O.lj_brute(ff, pos, types, box, 4)
    d = sphere - centre[:, None]
    assert np.array_equal(np.sum(d * d, axis=0) < rc * rc, delta < 0)   # the oracle's own pair set
    from paper_1001_3764_amd.md import MDSystem
    print("many cutoff pairs: precision=%s R=%d kernel=%d nl=%s" % (precision, R, kernel, nl), flush=True)
    kw = dict(nl_skin=1.0, nl_every=5, lj_kernel=kernel) if nl else dict(lj_kernel=kernel)
    s = MDSystem(ff, [pos.shape[1] // 4], box[None, :], [0.0], pos, np.zeros_like(pos), types, chain_len=4,
                 precision=precision, cell_div=R, **kw)
    # per-atom lists (kernel 4) hold 1.5x the mean neighbour count of this sparse box plus 64:
    # the centre's 100 partners overflow its list, so it walks its stencil instead
    flj = s.forces(lj_only=True)
    e = s.energies()[0]
    s.close()
    s6 = ff["sigma"][0] ** 6
    f_rc = 4 * ff["epsilon"][0] * (12 * s6 * s6 / rc ** 13 - 6 * s6 / rc ** 7)
    assert np.max(np.abs(flj - fo)) < 0.02 * abs(f_rc)
    _, eo = O.lj_brute(ff, pos, types, box, 4)
    assert e["e_lj"] == pytest.approx(eo["e_lj"], rel=1e-6)


def _ensemble(n_boxes=3):
    melts = [make_melt(c, density=0.80, T=300.0 + 50 * k, seed_melt=900 + k, seed_vel=950 + k, jitter=0.05)
             for k, c in enumerate((4, 11, 7)[:n_boxes])]
    return melts


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("kernel", [1, 2, 3, 6])
def test_batched_boxes(ff, precision, kernel):
    """Three boxes of different sizes in one context: bins, forces and a 10-step run of each
    box equal the box run alone (bit for bit) and match the oracle."""
    from paper_1001_3764_amd.md import MDSystem
    melts = _ensemble()
    pos = np.concatenate([m.pos for m in melts], axis=1)
    vel = np.concatenate([m.vel for m in melts], axis=1)
    types = np.concatenate([m.types for m in melts])
    T0 = [280.0, 0.0, 420.0]
    s = MDSystem(ff, [m.n_chains for m in melts], np.stack([m.box for m in melts]), T0, pos, vel, types,
                 precision=precision, cell_div=1, lj_kernel=kernel)
    start, atoms = s.bins()
    f_all = s.forces()
    s.step(10)
    p_all, v_all = s.state()
    e_all = s.energies()
    off = 0
    for b, m in enumerate(melts):
        n = m.n_atoms
        M, co, ao = s.grid(b)
        assert ao == off
        nc = int(np.prod(M))
        _, ostart, oatoms = O.bin_atoms(O.cell_index(m.pos, m.box, M), nc)
        np.testing.assert_array_equal(start[co:co + nc + 1] - start[co], ostart)
        np.testing.assert_array_equal(atoms[off:off + n] - off, oatoms)
        fo, _ = O.forces(ff, m.pos, m.types, m.box, 300)
        assert norm_err(f_all[:, off:off + n], fo) <= (TOL_FP64 if precision == "fp64" else TOL_MIXED)
        alone = MDSystem(ff, [m.n_chains], m.box[None, :], [T0[b]], m.pos, m.vel, m.types,
                         precision=precision, cell_div=1, lj_kernel=kernel)
        alone.step(10)
        p1, v1 = alone.state()
        assert np.array_equal(p1, p_all[:, off:off + n]) and np.array_equal(v1, v_all[:, off:off + n])
        e1 = alone.energies()[0]
        assert e1["e_kin"] == e_all[b]["e_kin"] and e1["e_lj"] == e_all[b]["e_lj"]
        alone.close()
        off += n
    s.close()


def test_error_paths(ff, melt):
    import paper_1001_3764_amd.md as md
    # box below 2R+1 cells: refused on the host at init
    small = make_melt(2, density=0.80, seed_melt=5)
    with pytest.raises(md.MDError) as ei:
        md.MDSystem(ff, [2], small.box[None, :], [0.0], small.pos, small.vel, small.types)
    assert ei.value.status == md.MD_ERR_BOX_TOO_SMALL
    # bad arguments
    with pytest.raises(md.MDError) as ei:
        md.MDSystem(dict(ff, rc=-1.0), [melt.n_chains], melt.box[None, :], [0.0], melt.pos, melt.vel,
                    melt.types)
    assert ei.value.status == md.MD_ERR_ARG
    # a non-finite coordinate is flagged by the device and the context refuses to step
    bad = melt.pos.copy()
    bad[1, 17] = np.nan
    s = md.MDSystem(ff, [melt.n_chains], melt.box[None, :], [0.0], bad, melt.vel, melt.types)
    with pytest.raises(md.MDError) as ei:
        s.energies()
    assert ei.value.status == md.MD_ERR_NONFINITE
    with pytest.raises(md.MDError) as ei:
        s.step(1)
    assert ei.value.status == md.MD_ERR_STATE
    s.close()


def test_runs_are_bitwise_reproducible(ff, melt):
    runs = []
    for _ in range(2):
        s = make_system(melt, ff, "mixed", 2, T0=350.0, lj_kernel=2)
        s.step(15)
        runs.append(s.state())
        s.close()
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_half_shell_repeats_bitwise_and_matches_full_shell(ff, melt, precision):
    """MD_LJ_HALFSHELL evaluates each pair once and adds both forces to int64 fixed-point
    accumulators.  Integer sums do not depend on the order of the atomics, so its forces repeat
    bit for bit across evaluations and contexts; they equal the full shell's to rounding."""
    from paper_1001_3764_amd.md import MD_LJ_HALFSHELL
    a = make_system(melt, ff, precision, 2, lj_kernel=MD_LJ_HALFSHELL)
    fa = a.forces(lj_only=True)
    ea = a.energies()[0]
    for _ in range(3):   # evaluate again: the accumulators were cleared after the last use
        a.compute_forces(with_energy=False)
    fa2 = a.forces(lj_only=True)
    c = make_system(melt, ff, precision, 2, lj_kernel=MD_LJ_HALFSHELL)
    fc = c.forces(lj_only=True)
    assert np.array_equal(fa, fa2) and np.array_equal(fa, fc)
    b = make_system(melt, ff, precision, 2, lj_kernel=2)
    fb = b.forces(lj_only=True)
    eb = b.energies()[0]
    tol = TOL_FP64 if precision == "fp64" else 2 * TOL_MIXED
    err = norm_err(fa, fb)
    print("half shell vs full shell (%s): %.3e" % (precision, err))
    assert err <= tol
    assert ea["e_lj"] == pytest.approx(eb["e_lj"], rel=1e-12 if precision == "fp64" else 2e-6)
    assert ea["virial"] == pytest.approx(eb["virial"], rel=1e-11 if precision == "fp64" else 2e-6)
    for s in (a, b, c):
        s.close()


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("kernel", [1, 2, 3, 6])
def test_pairs_at_the_cutoff_from_the_corners_of_a_home_group(ff, precision, kernel):
    """Four atoms in one cell (R = 2), at four corners of the box that bounds them, each with 7
    partners at r = rc (1 + delta), |delta| <= 4e-7, in directions pointing away from that box
    (well spaced: points of a 100-point Fibonacci sphere in that octant).
    There a partner's distance to the box equals its distance to the home: the tightest case
    for the cell tile's bounding-box filter, whose r^2 then equals the pair test's.  The LJ pair
    set must be the FP64 one, so every LJ force matches the oracle's far below |F(rc)|."""
    rc = ff["rc"]
    L = 60.0
    edge = L / np.floor(L * 2 / rc)
    lo, hi = 5 * edge + 0.3, 6 * edge - 0.3            # inside cell (5, 5, 5)
    homes = np.array([[lo, lo, lo], [hi, lo, lo], [lo, hi, lo], [lo, lo, hi]]).T
    outward = np.array([[-1, -1, -1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], float).T
    rng = np.random.default_rng(5)
    m = 100
    g = (1 + 5 ** 0.5) / 2
    t = np.arange(m) + 0.5
    sph = np.stack([np.cos(2 * np.pi * t / g) * np.sqrt(1 - (1 - 2 * t / m) ** 2),
                    np.sin(2 * np.pi * t / g) * np.sqrt(1 - (1 - 2 * t / m) ** 2), 1 - 2 * t / m])
    partners, deltas = [], []
    for k in range(4):
        inside = np.all(sph * outward[:, k:k + 1] >= 0.15, axis=0)
        u = sph[:, inside][:, :7]
        assert u.shape[1] == 7
        d = rng.uniform(1e-9, 4e-7, 7) * np.where(np.arange(7) % 2 == 0, 1.0, -1.0)
        partners.append(homes[:, k:k + 1] + rc * (1 + d) * u)
        deltas.append(d)
    # home chains: the home and three atoms far from everything else
    chains = []
    for k in range(4):
        far = np.array([[4.0 + 1.6 * j, 4.0 + 3.0 * k, 4.0] for j in range(3)]).T
        chains.append(np.concatenate([homes[:, k:k + 1], far], axis=1))
    pos = np.concatenate(chains + partners, axis=1)
    box = np.array([L, L, L])
    types = np.zeros(pos.shape[1], dtype=np.uint8)
    # the oracle's own decisions on the designed pairs: inside iff delta < 0
    for k in range(4):
        dd = partners[k] - homes[:, k:k + 1]
        assert np.array_equal(np.sum(dd * dd, axis=0) < rc * rc, deltas[k] < 0)
    fo, _ = O.lj_brute(ff, pos, types, box, 4)
    from paper_1001_3764_amd.md import MDSystem
    print("corner cutoff pairs: precision=%s kernel=%d" % (precision, kernel), flush=True)
    s = MDSystem(ff, [pos.shape[1] // 4], box[None, :], [0.0], pos, np.zeros_like(pos), types, chain_len=4,
                 precision=precision, cell_div=2, lj_kernel=kernel)
    M, _, _ = s.grid(0)
    assert np.all(M == 11)
    flj = s.forces(lj_only=True)
    s.close()
    s6 = ff["sigma"][0] ** 6
    f_rc = 4 * ff["epsilon"][0] * (12 * s6 * s6 / rc ** 13 - 6 * s6 / rc ** 7)
    assert np.max(np.abs(flj - fo)) < 0.02 * abs(f_rc)
