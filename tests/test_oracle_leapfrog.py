"""Pins of the oracle's leap-frog integrator, Nose-Hoover thermostat and centre-of-mass
velocity removal (Section 3 opening, Section 3.4; the COM-removal timing of Section 4).

What fixes them, other than the oracle itself:
  - with no thermostat, leap-frog and velocity Verlet generate the same positions, and the
    half-step velocity is the Verlet velocity half-kicked (a theorem about the two schemes);
  - with no forces, every velocity is scaled by the same factor each step, so the
    temperature and the friction follow the scalar system dT/dt = -2 xi T,
    dxi/dt = omega^2 (T/T0 - 1); the oracle must track its exact solution to second order
    in dt, and small oscillations of T have period tau / sqrt(2);
  - Nose-Hoover conserves KE + PE + dof R T0 (xi^2 / (2 omega^2) + eta); the discrete
    version to second order in dt;
  - removing the centre-of-mass velocity makes a run started with an extra uniform velocity
    w equal to the run without it, shifted by the one drift dt w taken before the removal.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle as O
from pe_melt import make_melt

ACC = 4.184e-4
RGAS = 1.987204259e-3


def free_gas(T, seed=0):
    """8 atoms on a 20 A lattice in a 40 A box: no pair within the cutoff, chain length 1
    (no bonded terms), so every force is zero."""
    g = np.array([(i, j, k) for i in (0, 1) for j in (0, 1) for k in (0, 1)], float).T * 20.0 + 5.0
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(3, 8)) * 0.01
    v -= v.mean(axis=1, keepdims=True)
    types = np.zeros(8, np.uint8)
    return g, v, types


def scale_to(ff, vel, types, T):
    _, t = O.kinetic(ff, vel, types)
    return vel * math.sqrt(T / t)


def min_image(d, box):
    return d - box[:, None] * np.round(d / box[:, None])


def test_leapfrog_without_thermostat_equals_velocity_verlet(ff):
    """v(-dt/2) = v(0) - dt/2 a(0): every position of the two schemes agrees, and the
    leap-frog velocity after n steps is v_VV(n) - dt/2 a(n)."""
    m = make_melt(1, density=0.02, jitter=0.05)
    dt, n = 1.0, 25
    mass = np.asarray(ff["mass"])[m.types]
    f0, _ = O.forces(ff, m.pos, m.types, m.box, 300)
    vh = m.vel - 0.5 * dt * ACC * f0 / mass
    for k in (1, 7, n):
        pv, vv, fv, _ = O.run(ff, m.pos, m.vel, f0, m.types, m.box, 300, k, dt=dt)
        pl, vl, fl, e = O.run_leapfrog(ff, m.pos, vh, f0, m.types, m.box, 300, k, dt=dt, T0=0.0)
        assert np.abs(min_image(pl - pv, m.box)).max() < 1e-11
        assert np.abs(vl - (vv - 0.5 * dt * ACC * fv / mass)).max() < 1e-13
        assert e["xi"] == 0.0 and e["eta"] == 0.0 and e["e_thermostat"] == 0.0


def nh_free_series(ff, dt, t_end, T_init, T0, tau):
    pos, vel, types = free_gas(T_init)
    vel = scale_to(ff, vel, types, T_init)      # taken as v(-dt/2)
    frc = np.zeros_like(pos)
    box = [40.0] * 3
    nh = (0.0, 0.0)
    Ts, xis = [], []
    for _ in range(int(round(t_end / dt))):
        pos, vel, frc, e = O.run_leapfrog(ff, pos, vel, frc, types, box, 1, 1, dt=dt, tau=tau, T0=T0, nh=nh)
        assert np.abs(frc).max() == 0.0
        nh = (e["xi"], e["eta"])
        Ts.append(e["temperature"])   # at t = (n + 1/2) dt
        xis.append(e["xi"])           # at t = (n + 1) dt
    return np.array(Ts), np.array(xis)


def test_nose_hoover_free_atoms_follow_the_equations_of_motion(ff):
    """No forces: T/T0 = y and xi obey dy/dt = -2 xi y, dxi/dt = omega^2 (y - 1), solved
    here by an adaptive integrator; the oracle's error is second order in dt."""
    T_init, T0, tau, t_end = 500.0, 300.0, 60.0, 240.0
    w2 = (2 * math.pi / tau) ** 2
    sol = solve_ivp(lambda t, s: [-2 * s[1] * s[0], w2 * (s[0] - 1)], (0.0, t_end + 1), [T_init / T0, 0.0],
                    rtol=1e-12, atol=1e-14, dense_output=True)
    errs = []
    for dt in (1.0, 0.5):
        Ts, xis = nh_free_series(ff, dt, t_end, T_init, T0, tau)
        n = np.arange(len(Ts))
        yT = sol.sol((n + 0.5) * dt)[0] * T0
        yxi = sol.sol((n + 1.0) * dt)[1]
        err = max(np.abs(Ts - yT).max() / T0, np.abs(xis - yxi).max() * tau)
        errs.append(err)
    assert errs[1] < 0.025             # 240 fs, two thermostat periods, dt = 0.5 fs
    assert 3.5 < errs[0] / errs[1] < 4.5     # second order


def test_nose_hoover_small_oscillation_period(ff):
    """Linearising about T = T0 gives u'' = -2 omega^2 u: T oscillates with period tau / sqrt(2)."""
    T0, tau, dt = 300.0, 40.0, 0.05
    Ts, _ = nh_free_series(ff, dt, 120.0, 1.002 * T0, T0, tau)
    t = (np.arange(len(Ts)) + 0.5) * dt
    u = Ts - T0
    k = np.where(np.sign(u[1:]) != np.sign(u[:-1]))[0]
    # linear interpolation of each crossing of T0
    tc = t[k] - u[k] * dt / (u[k + 1] - u[k])
    half_periods = np.diff(tc)
    assert len(half_periods) >= 4
    assert np.mean(half_periods) == pytest.approx(tau / math.sqrt(2) / 2, rel=2e-3)


def conserved_series(ff, m, dt, steps, T0, tau):
    """H(n+1) = KE(n+1) + PE(n+1) + E_thermostat(n+1), KE(n+1) the mean of the half-step
    kinetic energies on either side."""
    f, _ = O.forces(ff, m.pos, m.types, m.box, 300)
    mass = np.asarray(ff["mass"])[m.types]
    p, v = m.pos, m.vel - 0.5 * dt * ACC * f / mass
    nh = (0.0, 0.0)
    ke, rest = [], []
    for _ in range(steps):
        p, v, f, e = O.run_leapfrog(ff, p, v, f, m.types, m.box, 300, 1, dt=dt, tau=tau, T0=T0, nh=nh)
        nh = (e["xi"], e["eta"])
        ke.append(e["e_kin"])
        rest.append(e["e_lj_shifted"] + e["e_bond"] + e["e_angle"] + e["e_dih"] + e["e_thermostat"])
    ke = np.array(ke)
    H = 0.5 * (ke[:-1] + ke[1:]) + np.array(rest[:-1])
    return H, ke


def test_nose_hoover_extended_energy_is_conserved_to_second_order(ff):
    """One chain cooled from 500 K towards 300 K: the thermostat removes kinetic energy, the
    extended energy stays constant up to O(dt^2)."""
    m = make_melt(1, density=0.02, jitter=0.02, T=500.0)
    spans = []
    for dt, steps in ((1.0, 300), (0.5, 600)):
        H, ke = conserved_series(ff, m, dt, steps, 300.0, 100.0)
        spans.append(np.abs(H - H[0]).max())
        # the thermostat did work: the kinetic energy moved well beyond the error in H
        assert np.abs(ke - ke[0]).max() > 20 * spans[-1]
    assert 3.0 < spans[0] / spans[1] < 5.5


def test_com_removal_after_the_drift(ff):
    """A uniform extra velocity w: after the first step the run equals the run without it,
    displaced by dt w (the one drift taken before the removal), for both integrators."""
    m = make_melt(1, density=0.02, jitter=0.05, T=400.0)
    dt = 1.0
    w = np.array([0.003, -0.002, 0.0015])[:, None]
    f0, _ = O.forces(ff, m.pos, m.types, m.box, 300)
    for k in (1, 5, 20):
        a = O.run_leapfrog(ff, m.pos, m.vel, f0, m.types, m.box, 300, k, dt=dt, T0=350.0, remove_com=True)
        b = O.run_leapfrog(ff, m.pos, m.vel + w, f0, m.types, m.box, 300, k, dt=dt, T0=350.0, remove_com=True)
        assert np.abs(min_image(b[0] - a[0] - dt * w, m.box)).max() < 1e-10
        assert np.abs(b[1] - a[1]).max() < 1e-12
        assert b[3]["xi"] == pytest.approx(a[3]["xi"], rel=1e-9, abs=1e-15)
        assert np.abs(O.com_velocity(ff, b[1], m.types)).max() < 1e-16
        c = O.run(ff, m.pos, m.vel, f0, m.types, m.box, 300, k, dt=dt, T0=350.0, remove_com=True)
        d = O.run(ff, m.pos, m.vel + w, f0, m.types, m.box, 300, k, dt=dt, T0=350.0, remove_com=True)
        assert np.abs(min_image(d[0] - c[0] - dt * w, m.box)).max() < 1e-10
        assert np.abs(d[1] - c[1]).max() < 1e-12
    # without the removal the extra velocity stays
    e = O.run_leapfrog(ff, m.pos, m.vel + w, f0, m.types, m.box, 300, 5, dt=dt)
    assert np.abs(O.com_velocity(ff, e[1], m.types) - w[:, 0]).max() < 1e-12


def test_com_velocity_is_the_mass_weighted_mean(ff):
    rng = np.random.default_rng(5)
    v = rng.normal(size=(3, 50))
    types = (rng.random(50) < 0.3).astype(np.uint8)
    mass = np.asarray(ff["mass"])[types]
    np.testing.assert_allclose(O.com_velocity(ff, v, types), (v * mass).sum(axis=1) / mass.sum(), rtol=1e-13)
