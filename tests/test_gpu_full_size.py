"""GPU parity at the full sizes of the benchmark workloads, in the launch configuration the
benchmark times: mixed precision, autotuned stencil radius and LJ kernel, graph-replayed
steps.  The oracle computes sampled atoms one by one where the whole system would take too
long, and the whole system where it is cheap (bins, bonded terms, the smallest box)."""
import dataclasses
import os

import numpy as np
import pytest

import oracle as O
from pe_melt import WORKLOADS, build_melts

pytestmark = pytest.mark.gpu

TOL = 1e-5   # FP32 forces, norm-wise: max_i |F_gpu,i - F_ora,i| / F_rms(oracle)


def norm_err(d, frms):
    """max_i |d_i| / frms over atoms (columns)."""
    return float(np.max(np.sqrt(np.sum(d ** 2, axis=0))) / frms)


def rms(f):
    return float(np.sqrt(np.mean(np.sum(f ** 2, axis=0))))


def energy_close(e, ref, keys=("e_lj", "e_bond", "e_angle", "e_dih")):
    """Relative 2e-6 of the whole potential energy: a grown melt starts with every bond and
    angle at its minimum, where those terms are ~0 and a relative test of them alone is
    meaningless."""
    scale = sum(abs(ref[k]) for k in keys)
    for k in keys:
        assert e[k] == pytest.approx(ref[k], rel=2e-6, abs=2e-6 * scale), k


def threads():
    return max(1, min(16, os.cpu_count() or 1))


def system(ff, melts, wl, precision="mixed", **kw):
    from paper_1001_3764_amd.md import MDSystem
    pos = np.concatenate([m.pos for m in melts], axis=1)
    vel = np.concatenate([m.vel for m in melts], axis=1)
    types = np.concatenate([m.types for m in melts])
    boxes = np.stack([m.box for m in melts])
    print("system %s: %d boxes, N=%d, %s %s" % (wl.name, len(melts), pos.shape[1], precision, kw), flush=True)
    return MDSystem(ff, [m.n_chains for m in melts], boxes, list(wl.T0), pos, vel, types,
                    chain_len=wl.chain_len, dt=wl.dt_fs, tau=wl.tau_fs, precision=precision, **kw)


def check_bins(s, melt, b=0):
    M, cell_off, atom_off = s.grid(b)
    start, atoms = s.bins()
    nc = int(np.prod(M))
    cnt, ostart, oatoms = O.bin_atoms(O.cell_index(melt.pos, melt.box, M), nc)
    lo, hi = start[cell_off], start[cell_off + nc]
    np.testing.assert_array_equal(start[cell_off:cell_off + nc + 1] - lo, ostart)
    np.testing.assert_array_equal(atoms[lo:hi] - atom_off, oatoms)


def check_sampled_forces(ff, s, melt, n_sample, seed, atom_off=0, full=True):
    """Forces against the oracle at the same positions, norm-wise over the oracle's RMS force.
    full: the oracle's LJ force of every atom (so every atom is checked and F_rms is exact);
    otherwise its LJ force of n_sample uniformly drawn atoms, which also estimate F_rms, plus the
    50 atoms with the largest bonded force (checked, not used for F_rms).  Every bonded force
    is checked either way."""
    f = s.forces()[:, atom_off:atom_off + melt.n_atoms]
    flj = s.forces(lj_only=True)[:, atom_off:atom_off + melt.n_atoms]
    fo_b, _ = O.bonded(ff, melt.pos, melt.box, melt.chain_len)
    if full:
        fo_lj, _ = O.lj_cells(ff, melt.pos, melt.types, melt.box, melt.chain_len)
        frms = rms(fo_lj + fo_b)
        sample = np.arange(melt.n_atoms)
    else:
        rng = np.random.default_rng(seed)
        uniform = rng.choice(melt.n_atoms, size=n_sample, replace=False)
        top = np.argsort(np.sum(fo_b ** 2, axis=0))[-50:]   # forced contacts sit near them
        sample = np.unique(np.concatenate([uniform, top]))
        fo_lj, _ = O.lj_cells(ff, melt.pos, melt.types, melt.box, melt.chain_len, subset=sample)
        pos_u = np.searchsorted(sample, uniform)
        frms = rms(fo_lj[:, pos_u] + fo_b[:, uniform])
    err_lj = norm_err(flj[:, sample] - fo_lj, frms)
    err_b = norm_err(f - flj - fo_b, frms)
    err = norm_err(f[:, sample] - fo_lj - fo_b[:, sample], frms)
    print("force error over F_rms %.4f (%d atoms%s): LJ %.3e bonded %.3e total %.3e"
          % (frms, sample.size, "" if full else ", sampled", err_lj, err_b, err), flush=True)
    assert err_lj <= TOL and err_b <= TOL and err <= TOL


@pytest.fixture(scope="module")
def melt300k():
    O.set_threads(threads())
    return build_melts(WORKLOADS["melt300k_mixed"], threads())[0]


def test_melt300k_bins_forces_energies(ff, melt300k):
    """300,000 atoms: bins bit-exact, every bonded force, 4,000 sampled LJ forces, and the
    energies against the oracle's full sums."""
    s = system(ff, [melt300k], WORKLOADS["melt300k_mixed"], cell_div=0, lj_kernel=0, use_graph=True)
    print("tuned (R, kernel) =", s.tuning(), flush=True)
    check_bins(s, melt300k)
    check_sampled_forces(ff, s, melt300k, 4000, 17)   # every atom (full)
    e = s.energies()[0]
    _, eo = O.lj_cells(ff, melt300k.pos, melt300k.types, melt300k.box, 300)
    _, eb = O.bonded(ff, melt300k.pos, melt300k.box, 300)
    energy_close(e, {**eo, **eb})
    assert e["e_lj_shifted"] == pytest.approx(eo["e_lj_shifted"], rel=2e-6)
    s.close()


def test_melt300k_first_100_steps(ff, melt300k):
    """The Berendsen quench (500 -> 300 K), 100 graph-replayed steps: mixed and plain FP64 GPU
    forms against the oracle's own 100 steps."""
    wl = WORKLOADS["melt300k_mixed"]
    f0, _ = O.forces(ff, melt300k.pos, melt300k.types, melt300k.box, 300)
    po, vo, _, eo = O.run(ff, melt300k.pos, melt300k.vel, f0, melt300k.types, melt300k.box, 300, 100,
                          dt=wl.dt_fs, tau=wl.tau_fs, T0=wl.T0[0])
    out = {}
    for precision in ("mixed", "fp64"):
        s = system(ff, [melt300k], wl, precision, cell_div=0, lj_kernel=0, use_graph=True)
        s.step(100)
        p, v = s.state()
        T = s.energies()[0]["temperature"]
        s.close()
        d = p - po
        d -= melt300k.box[:, None] * np.round(d / melt300k.box[:, None])
        out[precision] = (float(np.abs(d).max()), float(np.abs(v - vo).max()), T)
        print("%s after 100 steps: max|dx| %.3e A, max|dv| %.3e A/fs, T %.6f (oracle %.6f)"
              % (precision, out[precision][0], out[precision][1], T, eo["temperature"]), flush=True)
    assert out["fp64"][0] <= 1e-8 and out["fp64"][2] == pytest.approx(eo["temperature"], rel=1e-10)
    assert out["mixed"][0] <= 1e-4 and out["mixed"][2] == pytest.approx(eo["temperature"], rel=1e-5)


def test_melt300k_leapfrog_nose_hoover_50_steps(ff, melt300k):
    """The paper's integrator at full size: leap-frog + Nose-Hoover (300 K, tau_T 100 fs) with
    the COM velocity removed every step, mixed precision, autotuned, graph-replayed, against
    the oracle's 50 steps."""
    wl = WORKLOADS["melt300k_mixed"]
    m = melt300k
    s = system(ff, [m], wl, "mixed", cell_div=0, lj_kernel=0, use_graph=True, integrator="leapfrog",
               remove_com=True)
    s.step(50)
    p, v = s.state()
    e = s.energies()[0]
    s.close()
    f0, _ = O.forces(ff, m.pos, m.types, m.box, 300)
    po, vo, _, eo = O.run_leapfrog(ff, m.pos, m.vel, f0, m.types, m.box, 300, 50, dt=wl.dt_fs, tau=wl.tau_fs,
                                   T0=wl.T0[0], remove_com=True)
    d = p - po
    d -= m.box[:, None] * np.round(d / m.box[:, None])
    print("leap-frog + NH after 50 steps: max|dx| %.3e A, max|dv| %.3e, xi %.9e (oracle %.9e), T %.6f (oracle %.6f)"
          % (np.abs(d).max(), np.abs(v - vo).max(), e["nh_xi"], eo["xi"], e["temperature"], eo["temperature"]),
          flush=True)
    assert np.abs(d).max() <= 1e-4
    assert e["temperature"] == pytest.approx(eo["temperature"], rel=1e-5)
    assert e["nh_xi"] == pytest.approx(eo["xi"], rel=1e-4)
    assert e["e_thermostat"] == pytest.approx(eo["e_thermostat"], rel=1e-4)


def test_melt300k_neighbour_lists_sampled_forces(ff, melt300k):
    """The list form as the benchmark runs it (skin 1 A, rebuilt every 10 steps, autotuned
    layout): 15 steps in, so the forces come from the refreshed payload between builds; every
    bonded force and 2,000 sampled LJ forces against the oracle at the current positions."""
    wl = WORKLOADS["melt300k_mixed"]
    s = system(ff, [melt300k], wl, cell_div=0, use_graph=True, nl_skin=1.0, nl_every=10)
    print("tuned (R, kernel) =", s.tuning(), flush=True)
    s.step(15)
    s.energies()   # raises MDError if the device flagged the list (an atom past half the skin, a full list)
    pos, _ = s.state()
    s.compute_forces(True)
    cur = dataclasses.replace(melt300k, pos=pos)
    check_sampled_forces(ff, s, cur, 2000, 31)
    s.energies()
    s.close()


def test_melt300k_half_shell_sampled_forces_and_energies(ff, melt300k):
    """The Newton-3 half shell (opt-in MD_LJ_HALFSHELL) as the benchmark runs it (R = 2, graph):
    every bonded force, 2,000 sampled LJ forces and the energies against the oracle; 10 steps in,
    bit-identical to a second context (integer sums do not depend on the order of the atomics)."""
    from paper_1001_3764_amd.md import MD_LJ_HALFSHELL
    wl = WORKLOADS["melt300k_mixed"]
    s = system(ff, [melt300k], wl, cell_div=2, lj_kernel=MD_LJ_HALFSHELL, use_graph=True)
    check_sampled_forces(ff, s, melt300k, 2000, 43)
    e = s.energies()[0]
    _, eo = O.lj_cells(ff, melt300k.pos, melt300k.types, melt300k.box, 300)
    _, eb = O.bonded(ff, melt300k.pos, melt300k.box, 300)
    energy_close(e, {**eo, **eb})
    t = system(ff, [melt300k], wl, cell_div=2, lj_kernel=MD_LJ_HALFSHELL, use_graph=True)
    s.step(10)
    t.step(10)
    ps, vs = s.state()
    pt, vt = t.state()
    assert np.array_equal(ps, pt) and np.array_equal(vs, vt)
    s.close()
    t.close()


def test_melt3M_bins_and_sampled_forces(ff):
    """3,000,000 atoms at 0.85 g/cm^3: bins bit-exact, every bonded force, 2,000 sampled LJ
    forces."""
    O.set_threads(threads())
    melt = build_melts(WORKLOADS["melt3M_mixed"], threads())[0]
    s = system(ff, [melt], WORKLOADS["melt3M_mixed"], cell_div=0, lj_kernel=0, use_graph=True)
    print("tuned (R, kernel) =", s.tuning(), flush=True)
    check_bins(s, melt)
    check_sampled_forces(ff, s, melt, 2000, 23)
    s.close()


def test_melt30M_bins_and_sampled_forces(ff):
    """The largest workload, 30,000,000 atoms (close to the 2^25 limit): bins bit-exact, every
    bonded force, 1,000 sampled LJ forces, in the benchmark's launch configuration."""
    O.set_threads(threads())
    melt = build_melts(WORKLOADS["melt30M_mixed"], threads())[0]
    s = system(ff, [melt], WORKLOADS["melt30M_mixed"], cell_div=0, lj_kernel=0, use_graph=True)
    print("tuned (R, kernel) =", s.tuning(), flush=True)
    check_bins(s, melt)
    check_sampled_forces(ff, s, melt, 4000, 29, full=False)
    s.step(2)
    e = s.energies()[0]
    assert np.isfinite(e["temperature"]) and e["step"] == 2
    s.close()


def test_ensemble64_smallest_box(ff):
    """The 64-box ensemble (about 4.3M atoms) in one launch sequence: every box's bins, and
    the smallest box's forces, energies and first 100 steps against the oracle."""
    O.set_threads(threads())
    wl = WORKLOADS["ensemble64_mixed"]
    melts = build_melts(wl, threads())
    s = system(ff, melts, wl, cell_div=0, lj_kernel=0, use_graph=True)
    print("tuned (R, kernel) =", s.tuning(), flush=True)
    for b, m in enumerate(melts):
        check_bins(s, m, b)
    b = int(np.argmin([m.n_atoms for m in melts]))
    m = melts[b]
    off = sum(x.n_atoms for x in melts[:b])
    f = s.forces()[:, off:off + m.n_atoms]
    fo, eo = O.forces(ff, m.pos, m.types, m.box, m.chain_len)
    err = norm_err(f - fo, rms(fo))
    print("smallest box %d (%d atoms): force error %.3e" % (b, m.n_atoms, err), flush=True)
    assert err <= TOL
    energy_close(s.energies()[b], eo)
    s.step(100)
    p, v = s.state()
    p, v = p[:, off:off + m.n_atoms], v[:, off:off + m.n_atoms]
    e100 = s.energies()
    s.close()
    po, vo, _, eo100 = O.run(ff, m.pos, m.vel, fo, m.types, m.box, m.chain_len, 100, dt=wl.dt_fs,
                             tau=wl.tau_fs, T0=wl.T0[b])
    d = p - po
    d -= m.box[:, None] * np.round(d / m.box[:, None])
    print("smallest box after 100 steps: max|dx| %.3e A, T %.6f (oracle %.6f)"
          % (np.abs(d).max(), e100[b]["temperature"], eo100["temperature"]), flush=True)
    assert np.abs(d).max() <= 1e-4
    assert e100[b]["temperature"] == pytest.approx(eo100["temperature"], rel=1e-5)


def test_melt300k_end_to_end_acf(ff, melt300k):
    """The end-to-end autocorrelation of the 1,000 chains after 20 graph-replayed steps against
    the oracle's, from the same positions (init is the reference)."""
    s = system(ff, [melt300k], WORKLOADS["melt300k_mixed"], cell_div=0, lj_kernel=0, use_graph=True)
    s.step(20)
    p, _ = s.state()
    got = s.ree_acf()[0]
    want = O.ree_acf(melt300k.pos, p, melt300k.box, 300)
    print("acf after 20 steps %.15f (oracle %.15f)" % (got, want), flush=True)
    assert got == pytest.approx(want, rel=0, abs=1e-12) and abs(got - 1.0) < 0.05
    s.close()
