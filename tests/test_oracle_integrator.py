"""Pins of the oracle's time integration (Section 3.4) and thermostat."""
import math

import numpy as np
import pytest

import oracle as O

ACC = 4.184e-4           # (kcal/mol/A)/(g/mol) in A/fs^2
RGAS = 1.987204259e-3


def test_harmonic_dimer_matches_discrete_verlet_solution(ff):
    """One CH2-CH2 bond, no LJ (1-2 excluded), no initial velocity.  The bond length obeys
    s'' = -w^2 s with w^2 = ACC kb / mu, and velocity Verlet gives exactly
    s_n = s_0 cos(n th) with cos(th) = 1 - (w dt)^2 / 2."""
    m = ff["mass"][0]
    mu = m / 2
    w = math.sqrt(ACC * ff["kb"] / mu)
    assert 2 * math.pi / w == pytest.approx(30.75, abs=0.01)      # period ~30.8 fs
    dt, s0 = 1.0, 0.05
    th = math.acos(1 - (w * dt) ** 2 / 2)
    pos = np.array([[20.0, 20.0 + ff["b0"] + s0], [20.0, 20.0], [20.0, 20.0]])
    vel = np.zeros((3, 2))
    types = np.zeros(2, np.uint8)
    box = [40.0] * 3
    frc, _ = O.forces(ff, pos, types, box, 2)
    for n in range(1, 121):
        pos, vel, frc, e = O.run(ff, pos, vel, frc, types, box, 2, 1, dt=dt)
        s = pos[0, 1] - pos[0, 0] - ff["b0"]
        assert s == pytest.approx(s0 * math.cos(n * th), abs=1e-12)
    assert np.abs(pos[1:] - 20.0).max() == 0.0


def test_time_reversibility(ff, melt3k):
    m = melt3k
    f0, _ = O.forces(ff, m.pos, m.types, m.box, 300)
    p, v, f, _ = O.run(ff, m.pos, m.vel, f0, m.types, m.box, 300, 20, dt=1.0)
    p2, v2, f2, _ = O.run(ff, p, -v, f, m.types, m.box, 300, 20, dt=1.0)
    d = p2 - m.pos
    d -= m.box[:, None] * np.round(d / m.box[:, None])
    assert np.abs(d).max() < 1e-9
    assert np.abs(v2 + m.vel).max() < 1e-10


def _isolated_gas(T, seed=0):
    """8 atoms on a 20 A lattice in a 40 A box: every pair beyond the cutoff, zero force."""
    g = np.array([(i, j, k) for i in (0, 1) for j in (0, 1) for k in (0, 1)], float).T * 20.0 + 5.0
    rng = np.random.default_rng(seed)
    types = np.zeros(8, np.uint8)
    v = rng.normal(size=(3, 8)) * 0.01
    v -= v.mean(axis=1, keepdims=True)
    return g, v, types


def test_berendsen_closed_form(ff):
    """With no forces, T_after_k = T0 + (1 - dt/tau)^k (T_init - T0) exactly."""
    pos, vel, types = _isolated_gas(500)
    box = [40.0] * 3
    _, t_init = O.kinetic(ff, vel, types)
    frc, _ = O.forces(ff, pos, types, box, 1)
    assert np.abs(frc).max() == 0.0
    dt, tau, T0 = 1.0, 100.0, 300.0
    for k in range(1, 60):
        pos, vel, frc, e = O.run(ff, pos, vel, frc, types, box, 1, 1, dt=dt, tau=tau, T0=T0)
        # reported temperature is the one the thermostat saw (before scaling)
        assert e["temperature"] == pytest.approx(T0 + (1 - dt / tau) ** (k - 1) * (t_init - T0), rel=1e-12)
        _, t_now = O.kinetic(ff, vel, types)
        assert t_now == pytest.approx(T0 + (1 - dt / tau) ** k * (t_init - T0), rel=1e-12)


def test_nve_without_thermostat_keeps_kinetic_energy_of_free_atoms(ff):
    pos, vel, types = _isolated_gas(500, seed=1)
    frc, _ = O.forces(ff, pos, types, [40.0] * 3, 1)
    k0, _ = O.kinetic(ff, vel, types)
    p, v, f, e = O.run(ff, pos, vel, frc, types, [40.0] * 3, 1, 25, T0=0.0)
    assert e["e_kin"] == pytest.approx(k0, rel=1e-15)
    np.testing.assert_allclose(p, pos + 25 * vel, rtol=0, atol=1e-12)


def test_velocity_verlet_positions_equal_leapfrog(ff):
    """The paper integrates with leap-frog; velocity Verlet generates the same positions."""
    from pe_melt import make_melt
    m = make_melt(1, density=0.02, jitter=0.05)        # one chain in a ~60 A box
    assert m.box[0] >= 3 * ff["rc"]
    dt, n = 1.0, 15
    mass = np.asarray(ff["mass"])[m.types]
    f0, _ = O.forces(ff, m.pos, m.types, m.box, 300)
    pv, vv, fv, _ = O.run(ff, m.pos, m.vel, f0, m.types, m.box, 300, n, dt=dt)
    # leap-frog: v(-dt/2) = v(0) - dt/2 a(0); v(t+dt/2) = v(t-dt/2) + dt a(t); x += dt v(t+dt/2)
    x = m.pos.copy()
    vh = m.vel - 0.5 * dt * ACC * f0 / mass
    f = f0
    for _ in range(n):
        vh = vh + dt * ACC * f / mass
        x = O.wrap(x + dt * vh, m.box)
        f, _ = O.forces(ff, x, m.types, m.box, 300)
    d = x - pv
    d -= m.box[:, None] * np.round(d / m.box[:, None])
    assert np.abs(d).max() < 1e-11


def test_energy_error_is_second_order(ff):
    """Total energy (shifted LJ + bonded + kinetic) fluctuates as O(dt^2) under NVE."""
    from pe_melt import make_melt
    m = make_melt(1, density=0.02, jitter=0.02, T=300.0)
    spans = []
    for dt, steps in ((1.0, 200), (0.5, 400)):
        f, e = O.forces(ff, m.pos, m.types, m.box, 300)
        ke, _ = O.kinetic(ff, m.vel, m.types)
        e0 = ke + e["e_lj_shifted"] + e["e_bond"] + e["e_angle"] + e["e_dih"]
        p, v = m.pos, m.vel
        dev = 0.0
        for _ in range(20):
            p, v, f, e = O.run(ff, p, v, f, m.types, m.box, 300, steps // 20, dt=dt)
            et = e["e_kin"] + e["e_lj_shifted"] + e["e_bond"] + e["e_angle"] + e["e_dih"]
            dev = max(dev, abs(et - e0))
        spans.append(dev)
    assert spans[0] < 0.05 * ke
    assert 2.5 < spans[0] / spans[1] < 6.0
