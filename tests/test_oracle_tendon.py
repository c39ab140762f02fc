"""Pins of the oracle's compliant-tendon step (CPU only).

The variant: a fibre with the damped force balance
F0 [a f_l(l) f_v(v) + f_p(l) + beta v] in series with a tendon linear above
its slack length (F0 at strain eps0); the series element acts on the
skeleton linearly implicitly in the new lengthening rate. Pinned against:
special values of the fibre-velocity root; a slide carrying a passive
Maxwell element, both against its hand-derived discrete recurrence and, at
first order in dt, against the matrix exponential of the continuous
system; the static balance of a fibre on a fixed path (Brent's method on
the balance equation); and the rigid step, which it must approach as the
tendon stiffens and the fibre damping vanishes.
"""
import numpy as np
import pytest
from scipy.linalg import expm
from scipy.optimize import brentq

from oracle import Oracle
from paper_2603_29332_amd import synth
from tests import models as tm

EPS0, BETA = 0.033, 0.1


@pytest.fixture(scope="module")
def lib():
    return Oracle(tm.maxwell_slide())


def test_fibre_velocity_root_special_values(lib):
    """Isometric balance (R = A) has the root 0; without activation the root
    is R / beta on either side; below the concentric limit (R <= -beta) the
    curve is zero and the root is R / beta; and the root inverts the curve
    on every branch."""
    for A in (0.0, 0.3, 1.0):
        for b in (0.01, 0.1, 1.0):
            assert abs(lib.fv_root(A, A, b)) < 1e-14
    for R in (-2.0, -0.05, 0.0, 0.4, 3.0):
        assert lib.fv_root(0.0, R, BETA) == pytest.approx(R / BETA, rel=1e-14, abs=1e-14)
    assert lib.fv_root(0.7, -0.5, BETA) == pytest.approx(-5.0, rel=1e-14)
    for A in (0.2, 0.9):
        for v in (-3.0, -1.0, -0.7, -0.2, -1e-3, 0.0, 1e-3, 0.05, 0.6, 4.0):
            R = A * lib.fv(v) + BETA * v
            assert lib.fv_root(A, R, BETA) == pytest.approx(v, abs=1e-12)
    rs = np.linspace(-1.0, 2.0, 301)
    roots = [lib.fv_root(0.8, R, BETA) for R in rs]
    assert np.all(np.diff(roots) > 0)


def _maxwell_constants(m):
    F0, lopt, ls, vmax = (float(np.float64(m[k][0])) for k in ("f0", "l_opt", "l_slack", "v_max"))
    k = F0 / (EPS0 * ls)                  # tendon stiffness, N/m
    b = F0 * BETA / (vmax * lopt)         # passive fibre damping, N s/m
    return F0, lopt, ls, k, b


def test_passive_maxwell_slide_follows_its_recurrence(lib):
    """Zero activation, fibre below its optimal length (no passive force):
    the muscle is a spring k in series with a damper b on a mass. Per step,
    with the tendon force F = k (L - l_m - l_s) and the fibre velocity
    v = F / b, the new velocity solves m (xd' - xd) = -dt (F + c (xd' - v))
    with c = k dt / (1 + k dt / b), then x' = x + dt xd' and
    l_m' = l_m + dt (v + c (xd' - v) / b)."""
    m = tm.maxwell_slide()
    o = lib
    F0, lopt, ls, k, b = _maxwell_constants(m)
    mass, d, dt = float(np.float32(2.0)), float(np.float32(0.28)), 1e-3
    x, xd, lm = 0.0, 0.3, 0.07              # tendon stretched 1 cm: F = 758 N
    q, qd, act, lmf = np.zeros(1), np.array([xd]), np.zeros(1), np.array([lm])
    for _ in range(200):
        q, qd, act, lmf, st = o.step_tendon(dt, q, qd, act, lmf, np.zeros(1), EPS0, BETA,
                                            contact=False)
        assert st == 0
        F = k * (d + x - lm - ls)
        assert F > 0                        # the tendon stays taut
        v = F / b
        c = k * dt / (1.0 + k * dt / b)
        xd = (mass * xd - dt * (F - c * v)) / (mass + dt * c)
        x = x + dt * xd
        lm = lm + dt * (v + c * (xd - v) / b)
        np.testing.assert_allclose([q[0], qd[0], lmf[0]], [x, xd, lm], rtol=1e-11, atol=1e-13)
    assert lmf[0] < lopt                    # no passive force throughout


def test_passive_maxwell_slide_converges_to_the_continuous_solution(lib):
    """The same system in continuous time: x' = xd, m xd' = -F,
    F' = k (xd - F / b); its solution at t = 0.05 s is expm(A t) y0. The
    step's error halves with dt (first order)."""
    m = tm.maxwell_slide()
    F0, lopt, ls, k, b = _maxwell_constants(m)
    mass, d = float(np.float32(2.0)), float(np.float32(0.28))
    x0, xd0, lm0 = 0.0, 0.3, 0.07
    A = np.array([[0.0, 1.0, 0.0], [0.0, 0.0, -1.0 / mass], [0.0, k, -k / b]])
    y0 = np.array([x0, xd0, k * (d + x0 - lm0 - ls)])
    T = 0.05
    yT = expm(A * T) @ y0
    errs = []
    for dt in (2e-4, 1e-4, 5e-5):
        q, qd, act, lmf = np.array([x0]), np.array([xd0]), np.zeros(1), np.array([lm0])
        for _ in range(int(round(T / dt))):
            q, qd, act, lmf, st = lib.step_tendon(dt, q, qd, act, lmf, np.zeros(1), EPS0, BETA,
                                                  contact=False)
            assert st == 0
        F = k * (d + q[0] - lmf[0] - ls)
        errs.append(np.abs(np.array([q[0], qd[0], F]) - yT) / np.array([1e-3, 1e-2, 10.0]))
    errs = np.array(errs).max(axis=1)
    assert errs[-1] < 0.2                     # close at the finest step
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 1.6 < r1 < 2.4 and 1.6 < r2 < 2.4


def test_fibre_on_a_fixed_path_relaxes_to_the_static_balance():
    """A muscle whose path length does not change, held at a constant
    excitation: the fibre relaxes until a f_l(l) + f_p(l) equals the tendon
    force F0 (L - l_m - l_s) / (l_s eps0) / F0 (Brent's method on that
    equation); the activation reaches the excitation."""
    m = tm.fixed_path_muscle()
    o = Oracle(m)
    lopt, ls = float(m["l_opt"][0]), float(m["l_slack"][0])
    L = float(o.geometry(np.zeros(1), np.zeros(1))[0][0])
    assert L == pytest.approx(0.31, abs=1e-7)
    for u in (0.0, 0.35, 1.0):
        q, qd, act, lmf = np.zeros(1), np.zeros(1), np.array([u]), np.array([L - ls - 1e-3])
        for _ in range(3000):
            q, qd, act, lmf, st = o.step_tendon(1e-3, q, qd, act, lmf, np.array([u]), EPS0, BETA,
                                                contact=False)
            assert st == 0
        def bal(lm):
            l = lm / lopt
            ft = max((L - lm - ls) / ls, 0.0) / EPS0
            return u * o.fl(l) + o.fp(l) - ft
        ls_static = brentq(bal, 0.3 * lopt, L - ls, xtol=1e-15)
        assert act[0] == pytest.approx(u, abs=1e-12)
        assert lmf[0] == pytest.approx(ls_static, abs=1e-10)
        assert q[0] == 0.0 and qd[0] == 0.0       # the path crosses no joint


def test_stiff_tendon_limit_is_the_rigid_step():
    """With a nearly rigid tendon stretched to carry the rigid model's force
    and a vanishing fibre damping, one compliant step equals the rigid step
    (the chain: 8 hinges, 16 muscles, random states and excitations)."""
    m = synth.chain_model(1)
    o = Oracle(m)
    nm = m["n_mus"]
    q0, qd0, a0 = synth.chain_initial_state(m, 6)
    u = synth.excitation_iid(5, 6, nm, 0)
    eps0, beta = 1e-8, 1e-9
    for e in range(6):
        q, qd, act = (np.asarray(v[e], np.float64) for v in (q0, qd0, a0))
        qr, qdr, ar, st, sg = o.step(1e-3, q, qd, act, u[e], contact=False, stages=True)
        assert st == 0
        # the tendon stretch that carries the rigid force at the step's start
        lm = sg["L"] - m["l_slack"] * (1.0 + eps0 * sg["F"] / m["f0"])
        qc, qdc, ac, lmc, st = o.step_tendon(1e-3, q, qd, act, lm, u[e], eps0, beta,
                                             contact=False)
        assert st == 0
        np.testing.assert_allclose(qdc, qdr, rtol=2e-6, atol=2e-6 * np.abs(qdr).max())
        np.testing.assert_allclose(qc, qr, rtol=0, atol=1e-3 * 2e-6 * np.abs(qdr).max() + 1e-12)
        np.testing.assert_array_equal(ac, ar)
        # the fibre followed the path: the tendon stays at its slack length
        Ln = o.geometry(qc, qdc)[0]
        np.testing.assert_allclose(Ln - lmc, m["l_slack"], rtol=0, atol=1e-8)


def test_recoil_through_the_slack_point_does_not_overshoot():
    """A passive fibre stretched to 1.5 optimal lengths behind a slack tendon
    recoils at several centimetres per second (f_p / beta) onto its static
    balance f_p(l) = f_t(L - l_m): the fibre length falls monotonically and
    never passes the balance (Brent's method), so the tendon never carries
    more than the balance force. An explicit step across the slack point
    would overshoot by up to dt times the recoil speed."""
    m = tm.fixed_path_muscle()
    o = Oracle(m)
    lopt, ls = float(m["l_opt"][0]), float(m["l_slack"][0])
    L = float(o.geometry(np.zeros(1), np.zeros(1))[0][0])
    q, qd, act, lmf = np.zeros(1), np.zeros(1), np.zeros(1), np.array([1.5 * lopt])
    assert lmf[0] + ls > L                   # slack at the start
    bal = lambda lm: o.fp(lm / lopt) - max((L - lm - ls) / ls, 0.0) / EPS0
    l_static = brentq(bal, 0.5 * lopt, 1.5 * lopt, xtol=1e-15)
    hist = [lmf[0]]
    for _ in range(400):
        q, qd, act, lmf, st = o.step_tendon(1e-3, q, qd, act, lmf, np.zeros(1), EPS0, BETA,
                                            contact=False)
        assert st == 0
        hist.append(lmf[0])
    hist = np.array(hist)
    assert np.all(np.diff(hist) <= 1e-15)
    assert hist.min() >= l_static - 1e-12
    assert hist[-1] == pytest.approx(l_static, abs=1e-10)
