"""Pins for the oracle's Table II material and contact model: the sigmoid
weight scaling muscle amplitude and phase (Sec. II-C with Table II's maximum
amplitude and phase), a dashpot beside every spring and a damped ground
(Table II damping ratios), and static/kinetic friction (Table II plane
coefficients).

Each feature is checked against a reduction of the system that does not go
through the oracle's force code: the single voxel's breathing mode, an
isolated node on the ground, the parallel combination of springs, conservation
laws, and central finite differences for the gradients."""
import cmath
import json
import math
import os

import numpy as np
import pytest

from paper_2405_00698_amd import inputs

QUIET = 1 | 2 | 4   # no gravity, no ground, no actuation
WACT = 8            # weight-scaled actuation


def _voxel(orc, c, w, **kw):
    return orc.Robot(1, np.array([c], np.uint8), np.array([w]), **kw)


def _damped_recurrence(n, delta, w2, gam, dt):
    """Closed form of u_{n+1} = u_n + dt r_{n+1}, r_{n+1} = r_n - dt (w2 u_n + gam r_n)
    from u_0 = delta, r_0 = 0: u_n = rho^n (A cos n th + B sin n th), with
    rho^2 = 1 - gam dt (the product of the two roots) and 2 rho cos th = 2 - gam dt - w2 dt^2
    (their sum); u_1 = (1 - w2 dt^2) delta fixes B."""
    rho = math.sqrt(1.0 - gam * dt)
    th = math.acos((2.0 - gam * dt - w2 * dt * dt) / (2.0 * rho))
    A = delta
    B = ((1.0 - w2 * dt * dt) * delta / rho - delta * math.cos(th)) / math.sin(th)
    return rho ** n * (A * math.cos(n * th) + B * math.sin(n * th))


def test_table2_preset_is_the_printed_table(orc):
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))
    t = orc.TABLE2
    ph, mat, pl = g["table_II_physics"], g["table_II_material"], g["table_II_plane"]
    assert t["gravity"] == ph["gravity_m_s2"] and t["mass"] == ph["mass_per_index_kg"]
    assert t["voxel_len"] == ph["original_rest_length_m"] and t["dt"] == ph["time_step_s"]
    assert t["k_class"][1] == t["k_class"][2] == mat["muscle_spring_constant_N_m"]
    assert t["k_class"][3] == mat["soft_tissue_spring_constant_N_m"]
    assert t["k_class"][4] == mat["hard_bone_spring_constant_N_m"]
    assert t["zeta_spring"] == mat["spring_damping_ratio"]
    assert abs(t["a_class"][1]) == abs(t["a_class"][2]) == mat["muscle_max_amplitude"]
    assert t["phi_class"][1] == t["phi_class"][2] == mat["muscle_max_phase_rad"]
    assert t["k_ground"] == pl["elastic_coefficient_N_m"] and t["zeta_ground"] == pl["damping_ratio"]
    assert t["mu_static"] == pl["static_friction"] and t["mu"] == pl["kinetic_friction"]
    assert t["flags"] & WACT


@pytest.mark.parametrize("c", [1, 2])
def test_weighted_actuation_single_voxel(orc, c):
    # one voxel: every spring has k = k_c w and k a e^{i phi} = k_c w (w a_c) e^{i w phi_c}
    w = 0.6
    R = _voxel(orc, c, w, **orc.TABLE2)
    sp = R.springs()
    kc, ac, pc = orc.TABLE2["k_class"][c], orc.TABLE2["a_class"][c], orc.TABLE2["phi_class"][c]
    np.testing.assert_allclose(sp["k"], kc * w, rtol=1e-15)
    Z = sp["k"] * sp["a"] * np.exp(1j * sp["phi"])
    np.testing.assert_allclose(Z, kc * w * (w * ac) * cmath.exp(1j * w * pc), rtol=1e-13)
    assert abs(sp["a"][0]) == pytest.approx(0.15, rel=1e-14)


def test_weighted_actuation_two_voxels_parallel(orc):
    """Two face-adjacent muscle voxels of different weights: the 6 springs of the
    shared face are two actuated springs in parallel, k1 (r - L1) + k2 (r - L2) =
    (k1 + k2)(r - L) with L = (k1 L1 + k2 L2) / (k1 + k2); checked at several
    times against the combined rest length the oracle's (k, a, phi) give."""
    cls = np.array([1, 1, 0, 0, 0, 0, 0, 0], np.uint8)
    w = np.array([0.3, 0.9, 0, 0, 0, 0, 0, 0])
    R = orc.Robot(2, cls, w, **orc.TABLE2)
    sp = R.springs()
    lat = R.node_lattice()
    xs = lat % 3
    shared = [s for s in range(R.S) if xs[sp["ij"][s, 0]] == 1 and xs[sp["ij"][s, 1]] == 1]
    assert len(shared) == 6
    kc, ac, pc = 2e3, 0.25, math.pi
    k1, k2 = kc * 0.3, kc * 0.9
    for s in shared:
        L0 = sp["L0"][s]
        for t in (0.0, 0.013, 0.071, 0.2):
            wt = 2 * math.pi * 4.0 * t
            L1 = L0 * (1 + 0.3 * ac * math.sin(wt + 0.3 * pc))
            L2 = L0 * (1 + 0.9 * ac * math.sin(wt + 0.9 * pc))
            L = L0 * (1 + sp["a"][s] * math.sin(wt + sp["phi"][s]))
            assert sp["k"][s] == pytest.approx(k1 + k2, rel=1e-15)
            assert L == pytest.approx((k1 * L1 + k2 * L2) / (k1 + k2), rel=1e-13, abs=1e-16)


def test_breathing_mode_weighted_actuation_with_phase(orc):
    # u'' = -(8k/m)(u - a sin(w t + phi)) with a = w a_c and phi = w phi_c
    wv, dt, delta = 0.7, 1e-4, 2e-3
    k, m = 2e3 * wv, 0.1
    R = _voxel(orc, 1, wv, **dict(orc.TABLE2, flags=WACT | 1 | 2, zeta_spring=0.0, zeta_ground=0.0, dt=dt))
    x, v, st, _ = R.state()
    c = x.mean(0)
    R.set_state(c + (1 + delta) * (x - c), v, st)
    r0 = x - c
    amp, ph = wv * 0.25, wv * math.pi
    u, r, ref = delta, 0.0, [delta]
    for n in range(1200):
        r = r + dt * (-8.0 * k / m * (u - amp * math.sin(2 * math.pi * 4.0 * n * dt + ph)))
        u = u + dt * r
        ref.append(u)
    for n in (1, 5, 300, 1200):
        R.step(n - R.state()[2])
        s = (R.state()[0] - c) / r0
        np.testing.assert_allclose(s - 1.0, ref[n], atol=1e-12)


def test_breathing_mode_spring_dashpot(orc):
    """Breathing by u: each spring stretches by u L0 at rate u' L0, so with dashpot
    c = zeta sqrt(2 m k) the corner force is -8 (k u + c u') (x_i0 - c): a damped
    scalar oscillator, w^2 = 8k/m and gam = 8c/m (modal damping ratio 2 zeta)."""
    k, m, dt, delta, zeta = 3e4, 0.1, 1e-4, 1e-2, 0.1   # bone of the base model
    R = _voxel(orc, 4, 1.0, flags=QUIET, damping=1.0, zeta_spring=zeta)
    x, v, st, _ = R.state()
    c = x.mean(0)
    R.set_state(c + (1 + delta) * (x - c), v, st)
    r0 = x - c
    w2, gam = 8 * k / m, 8 * zeta * math.sqrt(2 * m * k) / m
    for n in (1, 2, 50, 400, 1500):
        R.step(n - R.state()[2])
        s = (R.state()[0] - c) / r0
        np.testing.assert_allclose(s - 1.0, _damped_recurrence(n, delta, w2, gam, dt), atol=1e-13)
    # the envelope follows the continuous exp(-gam t / 2) to first order in dt
    n = 1500
    assert math.sqrt(1 - gam * dt) ** n == pytest.approx(math.exp(-gam * n * dt / 2), rel=0.02)


def test_dashpot_conserves_momentum(orc):
    # dashpot forces act in equal and opposite pairs along the spring: linear and
    # angular momentum stay constant without gravity, ground or velocity damping
    cls, w = inputs.random_voxels(3, 31, p_empty=0.2)
    R = orc.Robot(3, cls, w, flags=1 | 2, damping=1.0, zeta_spring=0.1)
    x, v, st, _ = R.state()
    v = np.random.default_rng(0).normal(0, 0.05, v.shape)
    R.set_state(x, v, st)
    P0, L0 = R.momentum()
    e0 = R.energy()
    R.step(3000)
    P1, L1 = R.momentum()
    np.testing.assert_allclose(P1, P0, atol=1e-14)
    np.testing.assert_allclose(L1, L0, atol=1e-14)
    # while the internal motion is damped out
    R2 = orc.Robot(3, cls, w, flags=1 | 2 | 4, damping=1.0, zeta_spring=0.1)
    R2.set_state(x, v - v.mean(0), st)
    e0 = R2.energy()
    R2.step(20000)
    assert R2.energy() < 0.05 * e0


def _free_nodes(orc, **kw):
    # a voxel whose class has zero stiffness: eight independent point masses
    kcl = (0.0, 0.0, 0.0, 0.0, 0.0)
    return _voxel(orc, 3, 1.0, **dict(dict(k_class=kcl, damping=1.0, flags=4), **kw))


def test_ground_damper_closed_form(orc):
    """A node resting in the penalty ground: d = z - z*, z* = -m g / k_c, obeys a
    damped oscillator with w^2 = k_c / m and gam = c_g / m = 2 zeta_g w; the
    amplitude is small enough that the normal force never reaches zero."""
    m, kg, g, dt, zg = 0.1, 1e5, 9.81, 1e-4, 0.1
    R = _free_nodes(orc, zeta_ground=zg)
    x, v, st, _ = R.state()
    zs = -m * g / kg
    x[:, 2] = 0.5 * zs
    R.set_state(x, np.zeros_like(v), st)
    w2, gam = kg / m, 2 * zg * math.sqrt(kg / m)
    for n in (1, 3, 60, 250):
        R.step(n - R.state()[2])
        z = R.state()[0][:, 2]
        np.testing.assert_allclose(z - zs, _damped_recurrence(n, 0.5 * zs - zs, w2, gam, dt), atol=1e-17)
    R.step(5000)
    np.testing.assert_allclose(R.state()[0][:, 2], zs, rtol=1e-9)


def test_ground_damper_never_pulls(orc):
    # a node leaving the ground fast: penalty 1e5 * 1e-7 = 0.01 N, damper
    # 2 * 0.1 * sqrt(1e5 * 0.1) * 1 m/s = 20 N, so the normal force is clamped to zero
    R = _free_nodes(orc, zeta_ground=0.1, flags=4)
    x, v, st, _ = R.state()
    x[:, 2] = -1e-7
    v[:, 2] = 1.0
    R.set_state(x, v, st)
    R.step(1)
    np.testing.assert_allclose(R.state()[1][:, 2], 1.0 - 9.81 * 1e-4, rtol=0, atol=1e-15)


@pytest.mark.parametrize("mu_s", [0.6, 1.5])
def test_static_and_kinetic_friction_block(orc, mu_s):
    """A node at the equilibrium depth (normal force m g) sliding at u0: each step
    removes mu_k g dt of speed, and the node sticks once the speed is within
    max(mu_s, mu_k) g dt.  With mu_s below mu_k (Table II's 0.6 and 1.0) the
    static coefficient never acts."""
    m, kg, g, dt, mu_k, u0 = 0.1, 1e5, 9.81, 1e-4, 1.0, 0.0129
    R = _free_nodes(orc, zeta_ground=0.1, mu=mu_k, mu_static=mu_s)
    x, v, st, _ = R.state()
    x[:, 2] = -m * g / kg
    v[:] = 0.0
    v[:, 0] = u0
    R.set_state(x, v, st)
    u, ref = u0, [u0]
    for n in range(20):
        u = 0.0 if u <= max(mu_s, mu_k) * g * dt else u - mu_k * g * dt
        ref.append(u)
    for n in range(1, 20):
        R.step(1)
        np.testing.assert_allclose(R.state()[1][:, 0], ref[n], atol=1e-12)
    # after 12 steps the speed (1.13e-3) lies between mu_k g dt and mu_s g dt
    assert (ref[13] > 0) if mu_s < mu_k else (ref[13] == 0.0)


def test_table2_friction_equals_single_kinetic_coefficient(orc):
    cls, w = inputs.random_voxels(3, 33, p_empty=0.2)
    params = dict(orc.TABLE2)
    A = orc.Robot(3, cls, w, **params)
    B = orc.Robot(3, cls, w, **dict(params, mu_static=0.0))
    A.step(3000)
    B.step(3000)
    np.testing.assert_array_equal(A.state()[0], B.state()[0])


def test_table2_robot_settles_and_moves(orc):
    # the full Table II model on a random 3^3 robot: finite, on the ground, and
    # the muscles move it
    cls, w = inputs.random_voxels(3, 34, p_empty=0.2)
    R = orc.Robot(3, cls, w, **orc.TABLE2)
    R.step(20000)
    x, v, st, dv = R.state()
    assert not dv and np.isfinite(x).all()
    assert x[:, 2].min() > -1e-3 and x[:, 2].min() < 1e-4
    assert abs(R.fitness()) > 1e-7


def _fd_check(R, n_steps, picks, tol=1e-3):
    sp = R.springs()
    J, gk, ga, gp = R.backward(n_steps)
    grads = {"k": gk, "a": ga, "phi": gp}
    for which in ("k", "a", "phi"):
        g = grads[which]
        scale = np.abs(g).max()
        for s in picks:
            eps = 1e-6 * abs(sp["k"][s]) if which == "k" else 1e-6
            vals = []
            for sign in (+1, -1):
                arr = {kk: sp[kk].copy() for kk in ("k", "a", "phi")}
                arr[which][s] += sign * eps
                R.set_springs(arr["k"], arr["a"], arr["phi"])
                vals.append(R.backward(n_steps)[0])
            R.set_springs(sp["k"], sp["a"], sp["phi"])
            fd = (vals[0] - vals[1]) / (2 * eps)
            assert abs(g[s] - fd) <= tol * max(abs(fd), 1e-3 * scale), (which, s, g[s], fd)


def test_adjoint_vs_fd_weighted_phase_and_static_friction(orc):
    # weight-scaled amplitude and phase (so phi != 0), static above kinetic
    # friction, contact; no dashpots (the adjoint does not cover them)
    cls, w = inputs.random_voxels(3, 35, p_empty=0.2)
    params = dict(orc.TABLE2, dt=1e-4, zeta_spring=0.0, zeta_ground=0.0, mu=0.5, mu_static=0.8, damping=0.999)
    R = orc.Robot(3, cls, w, **params)
    assert np.abs(R.springs()["phi"]).max() > 0.5
    _fd_check(R, 600, sorted(np.random.default_rng(3).choice(R.S, 6, replace=False)))


def test_adjoint_z_parametrisation_consistent(orc):
    # dJ/d(k, Zr, Zi) and dJ/d(k, a, phi) describe the same derivative:
    # with Z = k a e^{i phi}, dJ/da = k (cos phi dJ/dZr + sin phi dJ/dZi) and
    # dJ/dk|_{a,phi} = dJ/dk|_Z + a (cos phi dJ/dZr + sin phi dJ/dZi)
    cls, w = inputs.random_voxels(3, 36, p_empty=0.2)
    R = orc.Robot(3, cls, w, **dict(orc.TABLE2, dt=1e-4, zeta_spring=0.0, zeta_ground=0.0, damping=0.999))
    sp = R.springs()
    J, gk, ga, gp = R.backward(300)
    J2, gkz, gzr, gzi, gcd = R.backward_z(300)
    assert J == J2
    proj = np.cos(sp["phi"]) * gzr + np.sin(sp["phi"]) * gzi
    scale = np.abs(ga).max()
    np.testing.assert_allclose(ga, sp["k"] * proj, rtol=1e-9, atol=1e-12 * scale)
    np.testing.assert_allclose(gk, gkz + sp["a"] * proj, rtol=1e-9, atol=1e-12 * np.abs(gk).max())
    dphi = sp["k"] * sp["a"] * (np.cos(sp["phi"]) * gzi - np.sin(sp["phi"]) * gzr)
    np.testing.assert_allclose(gp, dphi, rtol=1e-9, atol=1e-12 * np.abs(gp).max())


def test_genome_gradient_vs_fd_weighted_actuation(orc):
    """dJ/dtheta when the weight also sets amplitude and phase: through
    d(k_c a_c w^2 e^{i w phi_c})/dw, the sigmoid head and the MLP."""
    B = inputs.gaussian_B().astype(np.float64)
    G = inputs.random_genomes(1, seed=5)[0].astype(np.float64)
    params = dict(orc.TABLE2, dt=1e-4, zeta_spring=0.0, zeta_ground=0.0, damping=0.999)
    n, steps = 3, 400
    J, g = orc.genome_fitness_grad(G, B, n, steps, **params)
    base_cls = orc.heads(orc.query(G, B, n))[0]
    assert np.isin(base_cls, [1, 2]).any()
    order = np.argsort(-np.abs(g))
    picks = list(order[:4]) + [inputs.OFF_B3 + 5, inputs.OFF_W2 + 130]
    for q in picks:
        vals = []
        for sign in (+1, -1):
            Gp = G.copy()
            Gp[q] += sign * 1e-6
            assert np.array_equal(orc.heads(orc.query(Gp, B, n))[0], base_cls)
            vals.append(orc.robot_from_genome(Gp, B, n, **params).backward(steps)[0])
        fd = (vals[0] - vals[1]) / 2e-6
        assert abs(g[q] - fd) <= 1e-3 * max(abs(fd), 1e-3 * np.abs(g).max()), (q, g[q], fd)


def test_adjoint_vs_fd_with_dashpots(orc):
    """Table II model in full: spring dashpots (zeta 0.1), the damped ground
    (zeta 0.1), weight-scaled muscles and static/kinetic friction; dJ/d(k, a,
    phi) against central differences on a 3^3 robot over 600 steps of contact."""
    cls, w = inputs.random_voxels(3, 38, p_empty=0.2)
    params = dict(orc.TABLE2, dt=1e-4, mu=0.5, mu_static=0.8, damping=1.0)
    R = orc.Robot(3, cls, w, **params)
    assert np.abs(R.dashpots()).min() > 0
    _fd_check(R, 600, sorted(np.random.default_rng(4).choice(R.S, 6, replace=False)))


def test_dashpot_coefficient_gradient_vs_fd(orc):
    """dJ/dc per spring dashpot coefficient against central differences
    (relative step 1e-6 of c)."""
    cls, w = inputs.random_voxels(3, 39, p_empty=0.2)
    R = orc.Robot(3, cls, w, **dict(orc.TABLE2, dt=1e-4, mu=0.5, damping=1.0))
    cd = R.dashpots()
    J, gc = R.backward_c(600)
    scale = np.abs(gc).max()
    assert scale > 0
    for s in sorted(np.random.default_rng(5).choice(R.S, 6, replace=False)):
        eps = 1e-6 * cd[s]
        vals = []
        for sign in (+1, -1):
            c2 = cd.copy()
            c2[s] += sign * eps
            R.dashpots(c2)
            vals.append(R.backward(600)[0])
        R.dashpots(cd)
        fd = (vals[0] - vals[1]) / (2 * eps)
        assert abs(gc[s] - fd) <= 1e-3 * max(abs(fd), 1e-3 * scale), (s, gc[s], fd)


def test_ground_damper_adjoint_vs_fd(orc):
    """The damped ground alone (no spring dashpots): its velocity term
    dN/dv_z = -c_g enters the velocity adjoint; checked through dJ/dk."""
    cls, w = inputs.random_voxels(3, 40, p_empty=0.2)
    R = orc.Robot(3, cls, w, **dict(orc.TABLE2, dt=1e-4, zeta_spring=0.0, zeta_ground=0.5, mu=0.5, damping=1.0))
    _fd_check(R, 600, sorted(np.random.default_rng(6).choice(R.S, 6, replace=False)))


def test_genome_gradient_vs_fd_with_dashpots(orc):
    """dJ/dtheta in the full Table II model: through the dashpot coefficient
    c = sum zeta sqrt(2 m k_c w) as well as k and Z, the sigmoid head and the
    MLP."""
    B = inputs.gaussian_B().astype(np.float64)
    G = inputs.random_genomes(1, seed=6)[0].astype(np.float64)
    params = dict(orc.TABLE2, dt=1e-4, damping=1.0)
    n, steps = 3, 400
    J, g = orc.genome_fitness_grad(G, B, n, steps, **params)
    base_cls = orc.heads(orc.query(G, B, n))[0]
    order = np.argsort(-np.abs(g))
    picks = list(order[:4]) + [inputs.OFF_B3 + 5, inputs.OFF_W2 + 130]
    for q in picks:
        vals = []
        for sign in (+1, -1):
            Gp = G.copy()
            Gp[q] += sign * 1e-6
            assert np.array_equal(orc.heads(orc.query(Gp, B, n))[0], base_cls)
            vals.append(orc.robot_from_genome(Gp, B, n, **params).backward(steps)[0])
        fd = (vals[0] - vals[1]) / 2e-6
        assert abs(g[q] - fd) <= 1e-3 * max(abs(fd), 1e-3 * np.abs(g).max()), (q, g[q], fd)


def test_dashpot_adjoint_reduces_to_base_without_dashpots(orc):
    """With zero damping ratios the dashpot terms vanish: the gradient equals
    the base-model adjoint of the same robot bit for bit, and dJ/dc is the
    derivative at c = 0 (nonzero: a dashpot would change the motion)."""
    cls, w = inputs.random_voxels(3, 41, p_empty=0.2)
    params = dict(orc.TABLE2, dt=1e-4, zeta_spring=0.0, zeta_ground=0.0, damping=0.999)
    R = orc.Robot(3, cls, w, **params)
    J, gk, ga, gp = R.backward(300)
    J2, gkz, gzr, gzi, gcd = R.backward_z(300)
    assert J == J2 and np.abs(gcd).max() > 0
    assert np.all(R.dashpots() == 0)
