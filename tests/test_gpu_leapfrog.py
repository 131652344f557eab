"""Leap-frog with the Nose-Hoover thermostat and centre-of-mass velocity removal (Section 3
opening, Section 3.4), through the C ABI, against the FP64 oracle."""
import numpy as np
import pytest

import oracle as O
from pe_melt import make_melt

pytestmark = pytest.mark.gpu

XTOL = {"fp64": 1e-9, "mixed": 1e-4}
RTOL = {"fp64": 1e-9, "mixed": 1e-5}
W = np.array([0.004, -0.0025, 0.0015])[:, None]   # uniform extra velocity, A/fs


@pytest.fixture(scope="module")
def melt():
    return make_melt(10, density=0.80, T=500.0, seed_melt=1000, seed_vel=1001, jitter=0.05)


def system(ff, m, precision, T0, vel=None, **kw):
    from paper_1001_3764_amd.md import MDSystem
    print("leapfrog system: N=%d %s T0=%s %s" % (m.n_atoms, precision, T0, kw), flush=True)
    return MDSystem(ff, [m.n_chains], m.box[None, :], [T0], m.pos, m.vel if vel is None else vel, m.types,
                    chain_len=m.chain_len, precision=precision, **kw)


def dx_max(p, q, box):
    d = p - q
    d -= box[:, None] * np.round(d / box[:, None])
    return float(np.abs(d).max())


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_leapfrog_nose_hoover_against_oracle(ff, melt, precision):
    """500 K melt with an extra uniform velocity, thermostatted towards 350 K (tau 100 fs)
    with the COM velocity removed every step: 100 steps checked every 25."""
    T0, tau = 350.0, 100.0
    v0 = melt.vel + W
    s = system(ff, melt, precision, T0, vel=v0, tau=tau, cell_div=0, lj_kernel=0, use_graph=True,
               integrator="leapfrog", remove_com=True)
    f0, _ = O.forces(ff, melt.pos, melt.types, melt.box, 300)
    p_o, v_o, f_o, nh = melt.pos, v0, f0, (0.0, 0.0)
    for chunk in range(4):
        s.step(25)
        p_o, v_o, f_o, e_o = O.run_leapfrog(ff, p_o, v_o, f_o, melt.types, melt.box, 300, 25, tau=tau, T0=T0,
                                            remove_com=True, nh=nh)
        nh = (e_o["xi"], e_o["eta"])
        p, v = s.state()
        e = s.energies()[0]
        print("%s after %d steps: max|dx| %.3e max|dv| %.3e xi %.9e (oracle %.9e) T %.6f (oracle %.6f)"
              % (precision, 25 * (chunk + 1), dx_max(p, p_o, melt.box), np.abs(v - v_o).max(), e["nh_xi"],
                 e_o["xi"], e["temperature"], e_o["temperature"]), flush=True)
        assert dx_max(p, p_o, melt.box) <= XTOL[precision]
        assert e["nh_xi"] == pytest.approx(e_o["xi"], rel=RTOL[precision] * 10)
        assert e["temperature"] == pytest.approx(e_o["temperature"], rel=RTOL[precision])
        assert e["e_kin"] == pytest.approx(e_o["e_kin"], rel=RTOL[precision])
        assert e["e_thermostat"] == pytest.approx(e_o["e_thermostat"], rel=RTOL[precision] * 10)
        assert e["e_lj"] == pytest.approx(e_o["e_lj"], rel=RTOL[precision] * 10)
    # the removal left no centre-of-mass motion
    assert np.abs(O.com_velocity(ff, v, melt.types)).max() < (1e-15 if precision == "fp64" else 1e-9)
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_verlet_berendsen_with_com_removal_against_oracle(ff, melt, precision):
    s = system(ff, melt, precision, 320.0, vel=melt.vel + W, cell_div=2, lj_kernel=2, remove_com=True)
    f0, _ = O.forces(ff, melt.pos, melt.types, melt.box, 300)
    s.step(50)
    po, vo, _, eo = O.run(ff, melt.pos, melt.vel + W, f0, melt.types, melt.box, 300, 50, T0=320.0,
                          remove_com=True)
    p, v = s.state()
    e = s.energies()[0]
    print("%s VV+COM after 50 steps: max|dx| %.3e T %.6f (oracle %.6f)"
          % (precision, dx_max(p, po, melt.box), e["temperature"], eo["temperature"]))
    assert dx_max(p, po, melt.box) <= XTOL[precision]
    assert e["temperature"] == pytest.approx(eo["temperature"], rel=RTOL[precision])
    assert e["nh_xi"] == 0.0 and e["e_thermostat"] == 0.0
    s.close()


def test_leapfrog_batched_boxes(ff):
    """Three boxes (one NVE) in one context: each against the oracle after 30 steps."""
    from paper_1001_3764_amd.md import MDSystem
    melts = [make_melt(c, density=0.80, T=300.0 + 60 * k, seed_melt=700 + k, seed_vel=750 + k, jitter=0.05)
             for k, c in enumerate((4, 9, 6))]
    T0 = [280.0, 0.0, 420.0]
    vel = [m.vel + (k + 1) * W for k, m in enumerate(melts)]
    s = MDSystem(ff, [m.n_chains for m in melts], np.stack([m.box for m in melts]), T0,
                 np.concatenate([m.pos for m in melts], axis=1), np.concatenate(vel, axis=1),
                 np.concatenate([m.types for m in melts]), precision="mixed", cell_div=2, lj_kernel=2,
                 use_graph=True, tau=80.0, integrator="leapfrog", remove_com=True)
    s.step(30)
    p_all, _ = s.state()
    es = s.energies()
    off = 0
    for b, m in enumerate(melts):
        fo, _ = O.forces(ff, m.pos, m.types, m.box, 300)
        po, _, _, eo = O.run_leapfrog(ff, m.pos, vel[b], fo, m.types, m.box, 300, 30, tau=80.0, T0=T0[b],
                                      remove_com=True)
        d = dx_max(p_all[:, off:off + m.n_atoms], po, m.box)
        print("box %d: max|dx| %.3e xi %.6e (oracle %.6e)" % (b, d, es[b]["nh_xi"], eo["xi"]))
        assert d <= XTOL["mixed"]
        assert es[b]["temperature"] == pytest.approx(eo["temperature"], rel=RTOL["mixed"])
        assert es[b]["nh_xi"] == pytest.approx(eo["xi"], rel=1e-4, abs=1e-12)
        off += m.n_atoms
    assert es[1]["nh_xi"] == 0.0 and es[1]["e_thermostat"] == 0.0
    s.close()


@pytest.mark.parametrize("nl", [False, True])
def test_leapfrog_graph_and_timed_steps_are_bit_identical(ff, melt, nl):
    kw = dict(cell_div=2, T0=330.0, vel=melt.vel + W, integrator="leapfrog", remove_com=True)
    if nl:
        kw.update(nl_skin=1.0, nl_every=4, lj_kernel=5)
    else:
        kw.update(lj_kernel=2)
    a = system(ff, melt, "mixed", use_graph=False, **kw)
    b = system(ff, melt, "mixed", use_graph=True, **kw)
    c = system(ff, melt, "mixed", use_graph=False, **kw)
    for n in (3, 7, 6):
        a.step(n)
        b.step(n)
        c.step_timed(n)
        pa, va = a.state()
        pb, vb = b.state()
        pc, vc = c.state()
        assert np.array_equal(pa, pb) and np.array_equal(va, vb)
        assert np.array_equal(pa, pc) and np.array_equal(va, vc)
    assert a.energies()[0] == b.energies()[0]
    for x in (a, b, c):
        x.close()


def test_leapfrog_neighbour_list_against_oracle(ff, melt):
    T0 = 350.0
    s = system(ff, melt, "mixed", T0, vel=melt.vel + W, cell_div=2, nl_skin=1.0, nl_every=5, lj_kernel=5,
               use_graph=True, integrator="leapfrog", remove_com=True)
    f0, _ = O.forces(ff, melt.pos, melt.types, melt.box, 300)
    s.step(40)
    po, _, _, eo = O.run_leapfrog(ff, melt.pos, melt.vel + W, f0, melt.types, melt.box, 300, 40, T0=T0,
                                  remove_com=True)
    p, _ = s.state()
    e = s.energies()[0]
    print("list + leap-frog after 40 steps: max|dx| %.3e" % dx_max(p, po, melt.box))
    assert dx_max(p, po, melt.box) <= XTOL["mixed"]
    assert e["nh_xi"] == pytest.approx(eo["xi"], rel=1e-4)
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_extended_energy_is_conserved(ff, melt, precision):
    """KE + PE + e_thermostat (KE at full steps as the mean of the half-step values) over 150
    steps of cooling from 500 K towards 300 K stays within 1% of the kinetic energy the
    thermostat removed, once the forced contacts of the grown melt have relaxed (20 steps;
    the FP64 oracle on the same run: 0.46%)."""
    s = system(ff, melt, precision, 300.0, cell_div=2, lj_kernel=2, use_graph=True, tau=100.0,
               integrator="leapfrog")
    ke, rest = [], []
    for _ in range(150):
        s.step(1)
        e = s.energies()[0]
        ke.append(e["e_kin"])
        rest.append(e["e_lj_shifted"] + e["e_bond"] + e["e_angle"] + e["e_dih"] + e["e_thermostat"])
    s.close()
    ke = np.array(ke)
    H = 0.5 * (ke[:-1] + ke[1:]) + np.array(rest[:-1])
    drift = np.abs(H[20:] - H[20]).max()
    removed = ke[0] - ke.min()
    print("%s: max|H - H(20)| %.4f kcal/mol, kinetic energy removed %.2f" % (precision, drift, removed))
    assert removed > 1000.0
    assert drift < 0.01 * removed
