"""The allocation-free set-up (md_init_system_static) against md_init_system with a caller
workspace: the same kernels on the same inputs, so bins, forces, energies and trajectories must
agree bit for bit.  Two allocation-free systems in a row, the second smaller, on the library's
one scratch array; the first is refused once the second has taken the array over."""
import numpy as np
import pytest

from pe_melt import make_melt

pytestmark = pytest.mark.gpu


def _pair(ff, m, static, **kw):
    from paper_1001_3764_amd.md import MDSystem
    print("system N=%d static=%s %s" % (m.n_atoms, static, kw), flush=True)
    return MDSystem(ff, [m.n_chains], m.box[None, :], [350.0], m.pos, m.vel, m.types, chain_len=m.chain_len,
                    precision=kw.pop("precision", "mixed"), cell_div=kw.pop("cell_div", 2),
                    lj_kernel=kw.pop("lj_kernel", 2), use_graph=False, static_workspace=static, **kw)


def _same(ref, sta, n_steps):
    rs, ra = ref.bins()
    ss, sa = sta.bins()
    assert np.array_equal(rs, ss) and np.array_equal(ra, sa)
    assert np.array_equal(ref.forces(), sta.forces())
    assert np.array_equal(ref.forces(lj_only=True), sta.forces(lj_only=True))
    assert ref.energies() == sta.energies()
    ref.step(n_steps)
    sta.step(n_steps)
    pr, vr = ref.state()
    ps, vs = sta.state()
    assert np.array_equal(pr, ps) and np.array_equal(vr, vs)
    assert ref.energies() == sta.energies()
    assert np.array_equal(ref.forces(), sta.forces())


def test_static_workspace_matches_caller_workspace(ff):
    from paper_1001_3764_amd.md import MD_ERR_STATE, MDError
    big = make_melt(10, density=0.80, T=500.0, seed_melt=1000, seed_vel=1001, jitter=0.05)
    small = make_melt(6, density=0.80, T=400.0, seed_melt=61, seed_vel=62, jitter=0.05)
    assert small.n_atoms < big.n_atoms
    ref1 = _pair(ff, big, False)
    sta1 = _pair(ff, big, True)
    _same(ref1, sta1, 20)
    ref1.close()
    # the second, smaller system takes the array over: the first can no longer run
    ref2 = _pair(ff, small, False, remove_com=True)
    sta2 = _pair(ff, small, True, remove_com=True)
    with pytest.raises(MDError) as ex:
        sta1.step(1)
    assert ex.value.status == MD_ERR_STATE
    sta1.close()
    _same(ref2, sta2, 25)
    ref2.close()
    sta2.close()


def test_static_workspace_fp64_neighbour_lists(ff):
    """FP64 with per-cell neighbour lists (their lists and build payload live in the array too)."""
    m = make_melt(6, density=0.80, T=400.0, seed_melt=61, seed_vel=62, jitter=0.05)
    ref = _pair(ff, m, False, precision="fp64", cell_div=2, lj_kernel=5, nl_skin=1.0, nl_every=5)
    sta = _pair(ff, m, True, precision="fp64", cell_div=2, lj_kernel=5, nl_skin=1.0, nl_every=5)
    _same(ref, sta, 12)
    ref.close()
    sta.close()
