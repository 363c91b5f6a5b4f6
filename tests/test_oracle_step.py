"""Pins for the oracle's time step, fitness and divergence handling.

The physics readings (Table II constants, semi-implicit Euler with all forces
from x_n, penalty ground, velocity-level Coulomb friction, per-step velocity
damping) are checked against closed forms and invariants that an independent
reduction of the system gives, not against the oracle's own formula."""
import math

import numpy as np
import pytest

from paper_2405_00698_amd import inputs

QUIET = 1 | 2 | 4   # no gravity, no ground, no actuation


def _cube(orc, c=4, w=1.0, **kw):
    return orc.Robot(1, np.array([c], np.uint8), np.array([w]), **kw)


def _breathe(R, delta):
    """Scale the single-voxel robot about its centre by (1 + delta)."""
    x, v, step, _ = R.state()
    c = x.mean(0)
    R.set_state(c + (1 + delta) * (x - c), v, step)
    return c, x - c


def _scalar_breathing(n_steps, delta, k, m, dt, damping=1.0, amp=0.0, freq=4.0):
    """The single voxel's breathing mode reduces to one scalar: x_i = c + s (x_i0 - c).
    Summing the 7 springs at each corner gives F_i = -8 k (s - 1 - a sin(w t_n)) (x_i0 - c),
    so u = s - 1 and its rate obey a scalar semi-implicit Euler recurrence."""
    u, w = delta, 0.0
    out = [u]
    for n in range(n_steps):
        acc = -8.0 * k / m * (u - amp * math.sin(2 * math.pi * freq * n * dt))
        w = damping * (w + dt * acc)
        u = u + dt * w
        out.append(u)
    return np.array(out)


def test_breathing_mode_discrete_closed_form(orc):
    k, m, dt, delta = 3e4, 0.1, 1e-4, 1e-2
    R = _cube(orc, c=4, w=1.0, flags=QUIET, damping=1.0)
    c, r0 = _breathe(R, delta)
    w2 = 8.0 * k / m
    th = math.acos(1.0 - w2 * dt * dt / 2.0)
    for n in (1, 7, 40, 333, 1000):
        R.step(n - R.state()[2])
        x = R.state()[0]
        s = (x - c) / r0
        u = delta * (math.cos(n * th) - w2 * dt * dt / (2 * math.sin(th)) * math.sin(n * th))
        np.testing.assert_allclose(s - 1.0, u, atol=1e-12)


def test_breathing_mode_actuated_and_damped(orc):
    # expanding muscle: rest length L0 (1 + 0.2 sin(2 pi 4 t)); damping 0.999 per step
    k, m, dt, delta = 1e4 * 0.7, 0.1, 1e-4, 3e-3
    R = _cube(orc, c=1, w=0.7, flags=1 | 2, damping=0.999)
    c, r0 = _breathe(R, delta)
    ref = _scalar_breathing(1500, delta, k, m, dt, damping=0.999, amp=0.2)
    for n in (1, 2, 100, 777, 1500):
        R.step(n - R.state()[2])
        s = (R.state()[0] - c) / r0
        np.testing.assert_allclose(s - 1.0, ref[n], atol=1e-11)
    # contracting muscle follows the opposite sign
    R = _cube(orc, c=2, w=0.7, flags=1 | 2, damping=0.999)
    c, r0 = _breathe(R, delta)
    ref = _scalar_breathing(600, delta, k, m, dt, damping=0.999, amp=-0.2)
    R.step(600)
    np.testing.assert_allclose((R.state()[0] - c) / r0 - 1.0, ref[600], atol=1e-11)


def test_rest_lattice_is_static(orc):
    cls, w = inputs.random_voxels(4, 7, p_empty=0.3)
    R = orc.Robot(4, cls, w, flags=QUIET)
    x0 = R.state()[0]
    R.step(1000)
    assert np.abs(R.state()[0] - x0).max() < 1e-12
    assert abs(R.fitness()) < 1e-12


@pytest.mark.parametrize("damping", [1.0, 0.999])
def test_momentum_decay_without_external_forces(orc, damping):
    cls, w = inputs.random_voxels(4, 3, p_empty=0.25)
    R = orc.Robot(4, cls, w, flags=1 | 2, damping=damping)
    x, v, step, _ = R.state()
    v = inputs.rng(5).normal(0, 0.05, v.shape)
    R.set_state(x, v, 0)
    P0, L0 = R.momentum()
    for n in (10, 500):
        R.step(n - R.state()[2])
        P, Lm = R.momentum()
        np.testing.assert_allclose(P, damping ** n * P0, atol=1e-13)
        np.testing.assert_allclose(Lm, damping ** n * L0, atol=1e-13)


def test_free_fall_of_com(orc):
    cls, w = inputs.random_voxels(3, 11, p_empty=0.2)
    R = orc.Robot(3, cls, w, flags=2, damping=1.0)     # gravity on, no ground, actuated
    z0 = R.state()[0][:, 2].mean()
    x0 = R.state()[0][:, 0].mean()
    g, dt = 9.81, 1e-4
    for n in (1, 50, 800):
        R.step(n - R.state()[2])
        x = R.state()[0]
        assert x[:, 2].mean() == pytest.approx(z0 - g * dt * dt * n * (n + 1) / 2, abs=1e-12)
        assert x[:, 0].mean() == pytest.approx(x0, abs=1e-12)


def test_energy_bounded_no_drift(orc):
    cls, w = inputs.random_voxels(2, 4, p_empty=0.0)
    R = orc.Robot(2, cls, w, flags=QUIET, damping=1.0)
    x, v, _, _ = R.state()
    R.set_state(x, inputs.rng(9).normal(0, 0.02, v.shape), 0)
    E = []
    for _ in range(200):
        R.step(100)
        E.append(R.energy())
    E = np.array(E)
    spread = E.max() - E.min()
    ke0 = 0.5 * 0.1 * (0.02 ** 2) * 3 * R.M
    assert spread < 0.2 * ke0                       # bounded oscillation, O(dt)
    slope = np.polyfit(np.arange(len(E)), E, 1)[0] * len(E)
    assert abs(slope) < 0.01 * ke0                  # no secular drift over 2e4 steps


def _settled_cube(orc, steps=30000, mu=0.5):
    R = _cube(orc, c=4, w=1.0, flags=4, damping=0.99, mu=mu)
    R.step(steps)
    return R


def test_ground_statics(orc):
    R = _settled_cube(orc)
    x = R.state()[0]
    m, g, kc = 0.1, 9.81, 1e5
    normal = kc * np.maximum(0.0, -x[:, 2])
    assert normal.sum() == pytest.approx(8 * m * g, rel=1e-9)
    bottom = x[:, 2] < 0.05
    np.testing.assert_allclose(x[bottom, 2], -2 * m * g / kc, rtol=1e-9)


def test_coulomb_sliding_block(orc):
    """Coulomb law at block level: while every contact node slides, friction
    removes dv_i = mu * dt * N_i / m from node i's horizontal slip along its
    direction, so the centre-of-mass x-velocity drops by sum_i dv_i * uhat_x,i / 8
    per step (the slip direction is that of the node's velocity after the step,
    since friction only shortens it).  The rigid-block deceleration mu g
    follows and the block comes to rest."""
    S = _settled_cube(orc, mu=0.0)   # no left-over lateral spring forces
    x = S.state()[0]
    R = _cube(orc, c=4, w=1.0, flags=4, damping=1.0)
    u0 = 0.05
    v = np.zeros_like(x)
    v[:, 0] = u0
    R.set_state(x, v, 0)
    mu, g, dt, m, kc = 0.5, 9.81, 1e-4, 0.1, 1e5
    prev = u0
    for n in range(1, 61):
        xp = R.state()[0]
        dv = mu * dt * kc * np.maximum(0.0, -xp[:, 2]) / m
        R.step(1)
        vn = R.state()[1]
        slip = np.hypot(vn[:, 0], vn[:, 1])
        assert np.all(slip[dv > 0] > 0)
        uhat_x = np.where(dv > 0, vn[:, 0] / np.where(slip > 0, slip, 1.0), 0.0)
        u = vn[:, 0].mean()
        assert prev - u == pytest.approx(np.sum(dv * uhat_x) / 8, rel=1e-8)
        prev = u
    assert prev == pytest.approx(u0 - 60 * mu * g * dt, rel=0.03)    # near-rigid block
    R.step(300)
    com = []
    for _ in range(200):
        R.step(1)
        com.append(R.state()[0][:, 0].mean())
    travel = np.array(com) - x[:, 0].mean()
    # stopped: the elastic block only rocks in place, having travelled forward
    # a distance of the order of the rigid block's u0^2 / (2 mu g)
    assert np.ptp(travel) < 1.5e-4
    assert 0.5 < travel.mean() / (u0 * u0 / (2 * mu * g)) < 1.0


def test_fitness_is_com_x_displacement(orc):
    cls, w = inputs.random_voxels(3, 2, p_empty=0.3)
    R = orc.Robot(3, cls, w)
    x, v, _, _ = R.state()
    R.set_state(x + np.array([0.37, -5.0, 2.0]), v, 0)
    assert R.fitness() == pytest.approx(0.37, abs=1e-14)
    x2 = x.copy()
    x2[0, 0] += 1.0
    R.set_state(x2, v, 0)
    assert R.fitness() == pytest.approx(1.0 / R.M, abs=1e-14)


def test_divergence_flag(orc):
    cls, w = inputs.random_voxels(3, 2, p_empty=0.3)
    R = orc.Robot(3, cls, w)
    R.set_springs(k=np.full(R.S, 1e12))
    R.step(200)
    assert R.state()[3] is True and R.fitness() == -math.inf
