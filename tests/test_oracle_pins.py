"""Pins of the FP64 oracle against closed forms, invariants, independent
routes and finite differences (CPU only).

Each pin is chosen so that a plausible slip in the oracle (a dropped term, a
wrong sign or index, a transposed operand) fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import Oracle
from paper_2603_29332_amd import synth
from tests import models as tm

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def f32(x):
    """Model constants are stored as float32: closed forms use the same
    rounded values."""
    return float(np.float32(x))


G = f32(9.81)


@pytest.fixture(scope="module")
def human():
    m = synth.human_model(2)
    return m, Oracle(m)


@pytest.fixture(scope="module")
def chain():
    m = synth.chain_model(1)
    return m, Oracle(m)


def _rand_pose(m, rng, spread=0.6):
    q = np.zeros(m["nq"])
    qd = rng.normal(size=m["nv"])
    if m["jtype"][0] == 2:
        q[:3] = rng.normal(size=3) * 0.3 + [0, 0, 1.0]
        xi = rng.normal(size=4)
        q[3:7] = xi / np.linalg.norm(xi)
        q[7:] = rng.uniform(-spread, spread, m["nq"] - 7)
    else:
        q[:] = rng.uniform(-spread, spread, m["nq"])
    return q, qd


def _qplus(m, q, v, h):
    """Move q along generalized velocity v for time h (exact for hinges;
    the free root's orientation by the quaternion exponential)."""
    qn = q.copy()
    if m["jtype"][0] != 2:
        return q + h * v
    qn[:3] += h * v[:3]
    th = v[3:6] * h
    a = np.linalg.norm(th)
    d = np.r_[np.cos(a / 2), np.sin(a / 2) * th / a] if a > 0 else np.r_[1, 0, 0, 0]
    x = q[3:7]
    qn[3:7] = np.r_[x[0] * d[0] - x[1:] @ d[1:],
                    x[0] * d[1:] + d[0] * x[1:] + np.cross(x[1:], d[1:])]
    qn[7:] += h * v[6:]
    return qn


# ----------------------------------------------------------- paper constants
def test_paper_constants_in_generator():
    """Activation time constants and the Hill parameter ranges used by the
    generator match the values the paper and the workload description fix."""
    g = json.load(open(os.path.join(GOLD, "paper_constants.json")))
    m = synth.chain_model(1)
    assert np.allclose(m["tau_act"], g["tau_act_s"]["value"])
    assert np.allclose(m["tau_deact"], g["tau_deact_s"]["value"])
    h = synth.human_model(2)
    assert h["n_mus"] == g["n_mtu"]["value"]
    assert h["nv"] == 80 and h["nq"] == 81
    assert abs(h["mass"].sum() - 75.0) < 1e-3
    assert (h["mass"] > 0).sum() == 22
    assert h["n_con"] == 24
    assert h["f0"].min() >= 200 and h["f0"].max() <= 1500


# ------------------------------------------------------- activation dynamics
def test_activation_rise_closed_form(chain):
    """u = 1: t(a) = tau_act [-2 ln((1-a)/(1-a0)) - 1.5 (a - a0)]; Euler
    converges to it at first order."""
    m, o = chain
    a0, a_target = 0.05, 0.6
    tau = 0.010
    t_exact = tau * (-2 * math.log((1 - a_target) / (1 - a0)) - 1.5 * (a_target - a0))
    errs = []
    for dt in (1e-5, 5e-6):
        a = np.full(m["n_mus"], a0)
        t = 0.0
        while a[0] < a_target:
            a_prev = a.copy()
            a = o.activation(dt, np.ones(m["n_mus"]), a)
            t += dt
        t_cross = t - dt + dt * (a_target - a_prev[0]) / (a[0] - a_prev[0])
        errs.append(abs(t_cross - t_exact))
    assert errs[0] < 2e-3 * t_exact
    assert 0.4 < errs[1] / errs[0] < 0.6     # first order in dt


def test_activation_decay_closed_form(chain):
    """u = 0: a/(0.5+1.5a) = a0/(0.5+1.5a0) exp(-t/(2 tau_deact))."""
    m, o = chain
    a0, T = 0.9, 0.05
    g = a0 / (0.5 + 1.5 * a0) * math.exp(-T / (2 * f32(0.040)))
    a_exact = 0.5 * g / (1 - 1.5 * g)
    errs = []
    for dt in (1e-5, 5e-6):
        a = np.full(m["n_mus"], a0)
        for _ in range(int(round(T / dt))):
            a = o.activation(dt, np.zeros(m["n_mus"]), a)
        errs.append(abs(a[0] - a_exact))
    assert errs[0] < 5e-4 * a_exact
    assert 0.4 < errs[1] / errs[0] < 0.6     # first order in dt


def test_activation_fixed_point_branch_and_clamp(chain):
    m, o = chain
    n = m["n_mus"]
    a = np.linspace(0, 1, n)
    assert np.array_equal(o.activation(2e-3, a, a), a)          # u = act
    # strict u > act uses tau_act: one step from 0 with u = 1
    up = o.activation(2e-3, np.ones(n), np.zeros(n))
    assert np.allclose(up, 2e-3 / (f32(0.010) * 0.5), rtol=1e-14)
    dn = o.activation(2e-3, np.zeros(n), np.ones(n))            # tau_deact/2
    assert np.allclose(dn, 1 - 2e-3 * 2.0 / f32(0.040), rtol=1e-14)
    # no overshoot (dt/tau <= 1) and clamping of u outside [0, 1]
    assert np.all(o.activation(2e-3, np.full(n, 5.0), np.zeros(n)) <= 1)
    assert np.array_equal(o.activation(2e-3, np.full(n, -3.0), a),
                          o.activation(2e-3, np.zeros(n), a))


# --------------------------------------------------------------- Hill curves
def test_hill_curve_special_values(chain):
    m, o = chain
    assert o.fl(1.0) == 1.0 and o.fv(0.0) == 1.0
    assert o.fv(-1.0) == 0.0 and o.fv(-3.0) == 0.0 and o.fp(1.0) == 0.0
    assert abs(o.fp(1.6) - 1.0) < 1e-12
    assert abs(o.fv(1e9) - 1.4) < 1e-6
    h = 1e-7
    for v in (0.0,):
        left = (o.fv(v) - o.fv(v - h)) / h
        right = (o.fv(v + h) - o.fv(v)) / h
        assert abs(left - 5.0) < 1e-5 and abs(right - 5.0) < 1e-5
    for v in (-0.7, -0.2, 0.05, 0.6):
        fd = (o.fv(v + h) - o.fv(v - h)) / (2 * h)
        assert abs(fd - o.fv_slope(v)) < 1e-6 * max(1, abs(fd))
    # f_l: symmetric about its maximum at l = 1, and its width fixed by the
    # Gaussian integral: the integral of exp(-(l-1)^2 / g) over the line is
    # sqrt(pi g), with g = 0.45 (reading R5)
    ls = np.linspace(1.0 - 8.0, 1.0 + 8.0, 160001)
    fl = np.array([o.fl(x) for x in ls])
    assert np.allclose(fl, fl[::-1], rtol=0, atol=1e-12)
    assert fl.argmax() == len(ls) // 2
    area = float(np.sum((fl[1:] + fl[:-1]) * 0.5 * np.diff(ls)))
    assert abs(area - np.sqrt(0.45 * np.pi)) < 1e-8
    # f_p continuous and C1 at 1.6 (linear tail)
    s_in = (o.fp(1.6) - o.fp(1.6 - h)) / h
    s_out = (o.fp(1.6 + h) - o.fp(1.6)) / h
    assert abs(s_in - s_out) < 1e-4 * s_in


def test_hill_force_isometric_optimal(chain):
    """F(act, l_m = 1, v = 0) = act F0, and F >= 0."""
    m, o = chain
    n = m["n_mus"]
    act = np.linspace(0, 1, n)
    L = m["l_slack"].astype(float) + m["l_opt"].astype(float)
    F = o.hill(act, L, np.zeros(n))
    assert np.allclose(F, act * m["f0"], rtol=1e-12)
    rng = np.random.default_rng(3)
    F2 = o.hill(rng.uniform(0, 1, n), L * rng.uniform(0.5, 2, n),
                rng.normal(size=n))
    assert np.all(F2 >= 0)


# ------------------------------------------------------------ muscle geometry
def test_two_point_muscle_law_of_cosines():
    """One hinge, origin on the ground at distance d1 from the axis, insertion
    on the link at distance d2: L^2 = d1^2 + d2^2 - 2 d1 d2 cos(phi),
    |r| = d1 d2 sin(phi) / L."""
    d1, d2 = f32(0.3), f32(0.25)
    m = tm.pendulum(muscles=[(800.0, 0.1, 0.2, [(-1, [0, 0, d1]), (0, [0, 0, -d2])])])
    o = Oracle(m)
    for q in (0.3, 1.0, 2.0, -1.2):
        L, r, Ld = o.geometry(np.array([q]), np.array([0.7]))
        phi = math.pi - abs(q)
        Lc = math.sqrt(d1 * d1 + d2 * d2 - 2 * d1 * d2 * math.cos(phi))
        assert abs(L[0] - Lc) < 1e-12
        assert abs(abs(r[0, 0]) - d1 * d2 * math.sin(phi) / Lc) < 1e-12
        # the path shortens as |q| grows toward pi: r has the sign of q
        assert np.sign(r[0, 0]) == np.sign(q)
        assert abs(Ld[0] + r[0, 0] * 0.7) < 1e-12


def test_moment_arms_match_finite_differences(human):
    m, o = human
    rng = np.random.default_rng(5)
    q, qd = _rand_pose(m, rng)
    L, r, Ld = o.geometry(q, qd)
    h = 1e-6
    for j in list(range(6)) + list(rng.choice(np.arange(6, m["nv"]), 10, replace=False)):
        e = np.zeros(m["nv"])
        e[j] = 1
        Lp, _, _ = o.geometry(_qplus(m, q, e, h), qd)
        Lm, _, _ = o.geometry(_qplus(m, q, e, -h), qd)
        assert np.abs((Lp - Lm) / (2 * h) + r[:, j]).max() < 1e-8
    assert np.abs(Ld + r @ qd).max() < 1e-12


def test_path_root_invariance_and_lower_bound(human):
    """L does not depend on the root pose; root moment arms are 0; the path
    is never shorter than its end-to-end distance."""
    m, o = human
    rng = np.random.default_rng(6)
    q, qd = _rand_pose(m, rng)
    L1, r1, _ = o.geometry(q, qd)
    q2 = q.copy()
    q2[:3] += [1.0, -2.0, 0.5]
    xi = rng.normal(size=4)
    q2[3:7] = xi / np.linalg.norm(xi)
    L2, _, _ = o.geometry(q2, qd)
    assert np.abs(L1 - L2).max() < 1e-12
    assert np.abs(r1[:, :6]).max() < 1e-12
    R, p = o.fk(q)
    vs, vn, vp = m["via_start"], m["via_node"], m["via_pos"].astype(float)
    for mu in range(0, m["n_mus"], 37):
        a, b = vs[mu], vs[mu + 1] - 1
        wa = R[vn[a]] @ vp[a] + p[vn[a]]
        wb = R[vn[b]] @ vp[b] + p[vn[b]]
        assert L1[mu] >= np.linalg.norm(wb - wa) - 1e-12


def test_moment_arm_sparsity_at_most_three_dofs(human):
    m, o = human
    rng = np.random.default_rng(7)
    q, qd = _rand_pose(m, rng)
    _, r, _ = o.geometry(q, qd)
    nz = (np.abs(r) > 1e-12).sum(axis=1)
    assert nz.max() <= 3 and nz.min() >= 1


def test_projection_is_virtual_work(human):
    """tau_j = sum_m r_mj F_m = -d(sum_m F_m L_m)/dq_j at frozen F."""
    m, o = human
    rng = np.random.default_rng(8)
    q, qd = _rand_pose(m, rng)
    _, r, _ = o.geometry(q, qd)
    F = rng.uniform(0, 1000, m["n_mus"])
    tau = r.T @ F
    h = 1e-6
    for j in rng.choice(np.arange(6, m["nv"]), 8, replace=False):
        e = np.zeros(m["nv"])
        e[j] = 1
        Lp, _, _ = o.geometry(_qplus(m, q, e, h), qd)
        Lm, _, _ = o.geometry(_qplus(m, q, e, -h), qd)
        assert abs(-(F @ Lp - F @ Lm) / (2 * h) - tau[j]) < 1e-6 * max(1, abs(tau[j]))


# -------------------------------------------------------------- mass matrix
def test_pendulum_mass_and_gravity():
    m_, d, Ic = 2.0, f32(0.4), f32(0.01)
    o = Oracle(tm.pendulum(m_, d, Ic))
    for q in (0.0, 0.7, -2.0):
        M = o.mass_matrix(np.array([q]))
        assert abs(M[0, 0] - (Ic + m_ * d * d)) < 1e-14
        C = o.bias(np.array([q]), np.array([3.0]))
        assert abs(C[0] - m_ * G * d * math.sin(q)) < 1e-12


def test_two_link_closed_form():
    """Spong's planar 2-link M and Coriolis terms."""
    m1, m2, l1, lc1, lc2, I1, I2 = map(f32, (1.5, 0.8, 0.5, 0.25, 0.2, 0.03, 0.01))
    o = Oracle(tm.two_link(m1, m2, l1, lc1, lc2, I1, I2))
    rng = np.random.default_rng(9)
    for _ in range(4):
        q = rng.uniform(-2, 2, 2)
        qd = rng.normal(size=2)
        c2, s2 = math.cos(q[1]), math.sin(q[1])
        M11 = I1 + I2 + m1 * lc1 ** 2 + m2 * (l1 ** 2 + lc2 ** 2 + 2 * l1 * lc2 * c2)
        M12 = I2 + m2 * (lc2 ** 2 + l1 * lc2 * c2)
        M22 = I2 + m2 * lc2 ** 2
        M = o.mass_matrix(q)
        assert np.allclose(M, [[M11, M12], [M12, M22]], atol=1e-13)
        hh = m2 * l1 * lc2 * s2
        Cv = np.array([-hh * (2 * qd[0] * qd[1] + qd[1] ** 2), hh * qd[0] ** 2])
        # hinges about +y with links along -z: angles grow toward +x
        Cg = o.bias(q, np.zeros(2))
        g = G
        th1 = q[0]
        th12 = q[0] + q[1]
        Gv = np.array([(m1 * lc1 + m2 * l1) * g * math.sin(th1) + m2 * lc2 * g * math.sin(th12),
                       m2 * lc2 * g * math.sin(th12)])
        assert np.allclose(Cg, Gv, atol=1e-12)
        assert np.allclose(o.rnea(q, qd, np.zeros(2), grav=False), Cv, atol=1e-12)


def test_mass_matrix_two_routes_and_spd(human):
    """Jacobian-sum M equals the RNEA-column M; M is symmetric positive
    definite."""
    m, o = human
    rng = np.random.default_rng(10)
    q, _ = _rand_pose(m, rng)
    nv = m["nv"]
    M = o.mass_matrix(q)
    C0 = o.rnea(q, np.zeros(nv), np.zeros(nv), grav=False)
    Mr = np.stack([o.rnea(q, np.zeros(nv), np.eye(nv)[j], grav=False) - C0
                   for j in range(nv)], 1)
    assert np.abs(Mr - M).max() < 1e-12 * np.abs(M).max()
    assert np.abs(M - M.T).max() < 1e-14 * np.abs(M).max()
    assert np.linalg.eigvalsh(M).min() > 0
    assert abs(M[0, 0] - 75.0) < 1e-4        # root translation sees all mass


def test_bias_skew_identity(human):
    """qd^T C_vel(q, qd) = 1/2 qd^T Mdot qd (Mdot by central differences)."""
    m, o = human
    rng = np.random.default_rng(11)
    q, qd = _rand_pose(m, rng)
    h = 1e-6
    Md = (o.mass_matrix(_qplus(m, q, qd, h)) - o.mass_matrix(_qplus(m, q, qd, -h))) / (2 * h)
    Cv = o.rnea(q, qd, np.zeros(m["nv"]), grav=False)
    assert abs(qd @ Cv - 0.5 * qd @ Md @ qd) < 1e-7 * max(1, abs(qd @ Cv))


def test_gravity_is_potential_gradient(human):
    """C(q, 0) with gravity equals dV/dq, V = -sum_b m_b g . c_b."""
    m, o = human
    rng = np.random.default_rng(12)
    q, _ = _rand_pose(m, rng)
    nv = m["nv"]
    Gq = o.bias(q, np.zeros(nv))
    h = 1e-6
    for j in [0, 1, 2, 3, 4, 5] + list(rng.choice(np.arange(6, nv), 8, replace=False)):
        e = np.zeros(nv)
        e[j] = 1
        Vp = o.energy(_qplus(m, q, e, h), np.zeros(nv))
        Vm = o.energy(_qplus(m, q, e, -h), np.zeros(nv))
        assert abs((Vp - Vm) / (2 * h) - Gq[j]) < 1e-6 * max(1, abs(Gq[j]))


# -------------------------------------------------------------------- solve
def test_cholesky_solve(human):
    m, o = human
    rng = np.random.default_rng(13)
    q, _ = _rand_pose(m, rng)
    M = o.mass_matrix(q)
    b = rng.normal(size=m["nv"])
    x, rc = o.chol_solve(M, b)
    assert rc == 0
    assert np.linalg.norm(M @ x - b) <= 1e-11 * np.linalg.norm(b) * np.linalg.cond(M) ** 0.5
    assert np.allclose(x, np.linalg.solve(M, b), rtol=1e-8, atol=1e-10)
    bad = np.array([[1.0, 2.0], [2.0, 1.0]])
    _, rc = o.chol_solve(bad, np.ones(2))
    assert rc == -1


# --------------------------------------------------------------- integrator
def _agm(a, b):
    for _ in range(60):
        a, b = 0.5 * (a + b), math.sqrt(a * b)
    return a


def test_pendulum_period_elliptic():
    """T = 4 sqrt(I_pivot/(m g d)) K(sin(theta0/2)), K by the AGM."""
    m_, d, Ic, th0 = 2.0, f32(0.4), f32(0.01), 1.2
    o = Oracle(tm.pendulum(m_, d, Ic))
    Ip = Ic + m_ * d * d
    k = math.sin(th0 / 2)
    K = math.pi / (2 * _agm(1.0, math.sqrt(1 - k * k)))
    T_exact = 4 * math.sqrt(Ip / (m_ * G * d)) * K
    errs = []
    for dt in (1e-3, 5e-4):
        q, qd = np.array([th0]), np.array([0.0])
        t, crossings = 0.0, []
        prev = q[0]
        while len(crossings) < 2:
            q, qd, _, st = o.step(dt, q, qd, np.zeros(0), np.zeros(0))
            assert st == 0
            t += dt
            if prev > 0 >= q[0]:
                crossings.append(t - dt + dt * prev / (prev - q[0]))
            prev = q[0]
        errs.append(abs((crossings[1] - crossings[0]) - T_exact))
    assert errs[0] < 2e-4 * T_exact
    assert errs[1] < 0.4 * errs[0]       # second order in dt


def test_energy_bounded_without_dissipation():
    """Symplectic Euler on the 8-link chain (no muscles, no damping): energy
    error stays O(dt) with no secular drift."""
    base = synth.chain_model(1)
    m = tm._base(list(base["parent"]), list(base["jtype"]), base["jpos"], base["axis"],
                 base["mass"], base["com"], base["inertia"])
    o = Oracle(m)
    q = np.full(8, 0.3)
    qd = np.zeros(8)
    E0 = o.energy(q, qd)
    dev = []
    for t in range(20000):
        q, qd, _, st = o.step(2e-4, q, qd, np.zeros(0), np.zeros(0))
        if t % 100 == 0:
            dev.append(o.energy(q, qd) - E0)
    dev = np.abs(np.array(dev))
    assert dev.max() < 1e-2 * abs(E0)
    assert dev[-50:].max() < 1.5 * dev[:150].max()     # no secular drift


def test_free_fall_exact_discrete():
    """Free root under gravity: p_n = p0 + n dt v0 - g dt^2 n(n+1)/2."""
    o = Oracle(tm.free_body())
    dt, n = 1e-3, 300
    q = np.array([0.1, -0.2, 5.0, 1, 0, 0, 0.0])
    v0 = np.array([0.5, 0.2, 1.0])
    qd = np.r_[v0, 0, 0, 0]
    for _ in range(n):
        q, qd, _, st = o.step(dt, q, qd, np.zeros(0), np.zeros(0))
    p = np.array([0.1, -0.2, 5.0]) + n * dt * v0 - np.array([0, 0, G]) * dt * dt * n * (n + 1) / 2
    assert np.abs(q[:3] - p).max() < 1e-12


def test_torque_free_spin_conserves_energy_and_momentum():
    o = Oracle(tm.free_body(gravity=(0, 0, 0)))
    I = np.array([0.02, 0.05, 0.08])
    q = np.array([0, 0, 0, 1, 0, 0, 0.0])
    w = np.array([0.3, 4.0, 0.2])
    qd = np.r_[0, 0, 0, w]

    def invariants(q, qd):
        x = q[3:7]
        R = np.array([[1 - 2 * (x[2] ** 2 + x[3] ** 2), 2 * (x[1] * x[2] - x[0] * x[3]), 2 * (x[1] * x[3] + x[0] * x[2])],
                      [2 * (x[1] * x[2] + x[0] * x[3]), 1 - 2 * (x[1] ** 2 + x[3] ** 2), 2 * (x[2] * x[3] - x[0] * x[1])],
                      [2 * (x[1] * x[3] - x[0] * x[2]), 2 * (x[2] * x[3] + x[0] * x[1]), 1 - 2 * (x[1] ** 2 + x[2] ** 2)]])
        wb = qd[3:6]
        return 0.5 * wb @ (I * wb), R @ (I * wb)
    E0, H0 = invariants(q, qd)
    for _ in range(2000):
        q, qd, _, _ = o.step(1e-4, q, qd, np.zeros(0), np.zeros(0))
    E1, H1 = invariants(q, qd)
    assert abs(E1 - E0) < 1e-3 * E0
    assert np.linalg.norm(H1 - H0) < 1e-3 * np.linalg.norm(H0)
    assert abs(np.linalg.norm(q[3:7]) - 1) < 1e-14


# ----------------------------------------------------- muscle equilibrium
def test_static_muscle_equilibrium():
    """One hinge, one muscle, gravity, qd = 0: with
    act* = (m g d sin q* / (r(q*) F0) - f_p(l_m)) / f_l(l_m) held by u = act*,
    qdd = 0 and the state stays put."""
    m_, d, Ic, F0 = 2.0, f32(0.4), f32(0.01), 1000.0
    pts = [(-1, [-0.05, 0, 0.3]), (0, [-0.03, 0, -0.25])]
    qs = 0.4
    probe = tm.pendulum(m_, d, Ic, muscles=[(F0, 0.1, 0.2, pts)])
    op = Oracle(probe)
    L, r, _ = op.geometry(np.array([qs]), np.array([0.0]))
    lopt = 0.1
    lsl = L[0] - 1.05 * lopt
    model = tm.pendulum(m_, d, Ic, muscles=[(F0, lopt, lsl, pts)])
    o = Oracle(model)
    L, r, _ = o.geometry(np.array([qs]), np.array([0.0]))
    lm = (L[0] - float(np.float32(lsl))) / float(np.float32(lopt))
    grav = m_ * G * d * math.sin(qs)
    act = (grav / (r[0, 0] * F0) - o.fp(lm)) / o.fl(lm)
    assert 0 < act < 1
    q, qd, a = np.array([qs]), np.array([0.0]), np.array([act])
    for _ in range(1000):
        q, qd, a, st = o.step(1e-3, q, qd, a, np.array([act]))
        assert st == 0
    assert abs(q[0] - qs) < 1e-12 and abs(qd[0]) < 1e-12


# ---------------------------------------------------------- implicit damping
def test_implicit_joint_damping_closed_form():
    """Pendulum without gravity and damping b: each step scales qd by
    I/(I + dt b) exactly."""
    Ic, d, m_, b, dt = f32(0.01), 0.0, 1.0, f32(0.3), 2e-3
    model = tm._base([-1], [0], [[0, 0, 0]], [[0, 1, 0]], [m_], [[0, 0, 0]],
                     [[Ic, Ic, Ic]], damping=[b], gravity=(0, 0, 0))
    o = Oracle(model)
    q, qd = np.array([0.0]), np.array([2.0])
    for n in range(1, 51):
        q, qd, _, _ = o.step(dt, q, qd, np.zeros(0), np.zeros(0))
    assert abs(qd[0] - 2.0 * (Ic / (Ic + dt * b)) ** 50) < 1e-13


def test_muscle_and_contact_slopes_match_finite_differences(human):
    """The implicit matrix D holds -d(tau)/d(qd) of the dissipative forces:
    compare its muscle part with central differences of J_m^T F in qd."""
    m, o = human
    rng = np.random.default_rng(14)
    q, _, _ = synth.human_initial_state(m, 1, seed=3)
    q = q[0].astype(float)
    qd = rng.normal(size=m["nv"]) * 0.5
    u = rng.uniform(0, 1, m["n_mus"])
    act = rng.uniform(0, 1, m["n_mus"])
    dt = 1e-3
    _, _, _, _, S = o.step(dt, q, qd, act, u, contact=False, stages=True)
    D = S["D"] - np.diag(m["damping"].astype(float))
    act1 = S["act"]
    h = 1e-6
    for j in rng.choice(np.arange(6, m["nv"]), 6, replace=False):
        e = np.zeros(m["nv"])
        e[j] = h
        Lp, rp, Ldp = o.geometry(q, qd + e)
        Lm, rm, Ldm = o.geometry(q, qd - e)
        tp = rp.T @ o.hill(act1, Lp, Ldp)
        tmn = rm.T @ o.hill(act1, Lm, Ldm)
        col = -(tp - tmn) / (2 * h)
        assert np.abs(col - D[:, j]).max() < 1e-5 * max(1, np.abs(D[:, j]).max())
    # contact slope: point mass on the ground, sliding
    pm = tm.point_mass_slides()
    op = Oracle(pm)
    qc = np.array([0.0, 0.0, 0.015])
    qdc = np.array([0.05, -0.03, -0.02])
    dtc = 1e-3
    _, _, Dc = op.contact(qc, qdc, dtc, with_slope=True)
    for j in range(3):
        e = np.zeros(3)
        e[j] = 1e-7
        tp, _ = op.contact(qc, qdc + e, dtc)
        tn, _ = op.contact(qc, qdc - e, dtc)
        fd = -(tp - tn) / 2e-7
        if j < 2:
            assert np.allclose(fd[:2], Dc[:2, j], rtol=1e-5)
            # the normal force does not depend on the tangential velocity
            assert abs(fd[2]) < 1e-9 and Dc[2, j] == 0.0
        else:
            # normal slope: damping plus the implicit spring, c_d + dt k
            assert abs(fd[2] - Dc[2, 2]) < 1e-4 * Dc[2, 2]
            # the friction slope is taken at fixed F_n (reading R15): the
            # true cross term through F_n's damping is left out of D
            assert np.all(Dc[:2, 2] == 0.0) and np.abs(fd[:2]).max() > 1.0
    assert abs(Dc[2, 2] - (1e3 + dtc * 1e5)) < 1e-9


# ------------------------------------------------------------------- contact
def test_contact_resting_penetration():
    """A resting point mass settles at penetration m g / k."""
    m_ = 1.5
    o = Oracle(tm.point_mass_slides(m=m_))
    q, qd = np.array([0.0, 0.0, 0.02]), np.zeros(3)
    for _ in range(3000):
        q, qd, _, st = o.step(1e-3, q, qd, np.zeros(0), np.zeros(0))
        assert st == 0
    pen = 0.02 - q[2]
    assert abs(pen - m_ * G / 1e5) < 1e-9
    tau, n = o.contact(q, np.zeros(3), 1e-3)
    assert n == 1 and abs(tau[2] - m_ * G) < 1e-6


def test_contact_sliding_stops_near_coulomb_distance():
    """A fast slide decelerates at about mu g: stopping distance v0^2/(2 mu g)
    (the regularisation leaves a small creep)."""
    m_ = 1.5
    o = Oracle(tm.point_mass_slides(m=m_))
    pen = m_ * G / 1e5
    q, qd = np.array([0.0, 0.0, 0.02 - pen]), np.array([3.0, 0.0, 0.0])
    for _ in range(2000):
        q, qd, _, _ = o.step(1e-3, q, qd, np.zeros(0), np.zeros(0))
    d_exact = 3.0 ** 2 / (2 * G)
    assert abs(q[0] - d_exact) < 0.05 * d_exact
    assert abs(qd[0]) < 0.05


# ---------------------------------------------------------- given geometry
def test_given_geometry_step_matches_computed(human):
    """The step with geometry supplied (the surrogate's entry into the
    dynamics) reduces to the ordinary step when the supplied values are the
    exact path geometry, and a length change of one muscle moves only that
    muscle's Hill force, by the Hill law."""
    m, o = human
    rng = np.random.default_rng(21)
    q, qd = _rand_pose(m, rng, 0.3)
    qd *= 0.3
    act = rng.uniform(0.05, 0.9, m["n_mus"])
    u = rng.uniform(0, 1, m["n_mus"])
    L, r, _ = o.geometry(q, qd)
    a = o.step(1e-3, q, qd, act, u, stages=True)
    b = o.step(1e-3, q, qd, act, u, stages=True, geometry=(L, r))
    for x, y in zip(a[:3], b[:3]):
        assert np.abs(x - y).max() < 1e-12
    assert a[3] == b[3] == 0
    k = 17
    L2 = L.copy()
    L2[k] += 0.004
    c = o.step(1e-3, q, qd, act, u, stages=True, geometry=(L2, r))
    dF = c[4]["F"] - a[4]["F"]
    assert np.abs(np.delete(dF, k)).max() == 0.0
    Fk = o.hill(c[4]["act"], L2, a[4]["Ldot"])[k]
    assert abs(c[4]["F"][k] - Fk) < 1e-12 * max(1.0, abs(Fk))
    assert abs(dF[k]) > 0
