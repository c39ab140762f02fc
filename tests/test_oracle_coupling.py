"""Pins of the oracle's joint coupling (anatomical equality constraints as a
penalty, Methods, "GPU-accelerated simulation framework"): the force is
minus the gradient of the spring energy k/2 sum phi^2 plus the damper, its
velocity slope D is (d + dt k) J^T J (central differences), and as the
stiffness grows the oracle's step approaches the exactly constrained
dynamics computed by a second route, the null-space (reduced-coordinate)
equations of motion."""
import numpy as np
import pytest

from oracle import Oracle
from paper_2603_29332_amd import synth

DT = 1e-3


def _chain_coupled(k, d, ratio=0.5):
    m = dict(synth.chain_model(1))
    m["n_eq"] = 1
    m["eq_start"] = np.array([0, 2], np.int32)
    m["eq_dof"] = np.array([5, 2], np.int32)        # q5 follows ratio * q2 (q2 is q5's ancestor)
    m["eq_coef"] = np.array([1.0, -ratio], np.float32)
    m["eq_off"] = np.zeros(1, np.float32)
    m["eq_k"], m["eq_d"] = np.float32(k), np.float32(d)
    return m


def test_coupling_force_is_the_spring_gradient_plus_damper():
    rng = np.random.default_rng(0)
    m = _chain_coupled(300.0, 7.0)
    o = Oracle(m)
    nv = m["nv"]
    q = rng.uniform(-0.4, 0.4, m["nq"])
    qd = rng.uniform(-1, 1, nv)
    tau, D, phi = o.coupling(q, qd, DT)
    J = np.zeros((1, nv))
    J[0, 5], J[0, 2] = 1.0, -0.5
    assert np.allclose(phi, J @ q, rtol=0, atol=1e-15)
    # velocity slope by central differences (tau is linear in qd)
    h = 1e-3
    Dfd = np.zeros((nv, nv))
    for j in range(nv):
        e = np.zeros(nv)
        e[j] = h
        Dfd[:, j] = -(o.coupling(q, qd + e, DT)[0] - o.coupling(q, qd - e, DT)[0]) / (2 * h)
    assert np.abs(Dfd - D).max() < 1e-9 * np.abs(D).max()
    assert np.allclose(D, (7.0 + DT * 300.0) * J.T @ J, rtol=1e-12, atol=0)
    # position part: -d tau/dq = k J^T J, the Hessian of k/2 phi^2
    Kfd = np.zeros((nv, nv))
    for j in range(nv):
        e = np.zeros(nv)
        e[j] = h
        Kfd[:, j] = -(o.coupling(q + e, qd, DT)[0] - o.coupling(q - e, qd, DT)[0]) / (2 * h)
    assert np.allclose(Kfd, 300.0 * J.T @ J, rtol=1e-9, atol=1e-9)
    # and the force itself
    deff = 7.0 + DT * 300.0
    assert np.allclose(tau, -J.T @ (300.0 * (J @ q) + deff * (J @ qd)), rtol=1e-12, atol=1e-12)


def test_no_coupling_leaves_the_step_unchanged():
    base = synth.chain_model(1)
    m = _chain_coupled(0.0, 0.0)
    rng = np.random.default_rng(1)
    q = rng.uniform(-0.3, 0.3, base["nq"])
    qd = rng.uniform(-1, 1, base["nv"])
    act = rng.uniform(0, 0.5, base["n_mus"])
    u = rng.uniform(0, 1, base["n_mus"])
    a = Oracle(base).step(DT, q, qd, act, u, contact=False)
    b = Oracle(m).step(DT, q, qd, act, u, contact=False)
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)


def _nullspace_qdd(m, q, qd, act, u):
    """Constrained acceleration by the reduced-coordinate route: with
    q = T z (the coupled DoF eliminated), qdd = T (T^T H T)^-1 T^T rhs, H and
    rhs the oracle's own unconstrained step matrix and right-hand side."""
    mu = dict(m)
    mu["n_eq"] = 0
    ou = Oracle(mu)
    _, _, _, st, S = ou.step(DT, q, qd, act, u, contact=False, stages=True)
    nv = m["nv"]
    H = S["M"] + DT * S["D"]
    rhs = S["tau_mus"] + S["tau_ext"] + S["tau_d"] - S["C"]
    T = np.delete(np.eye(nv), 5, axis=1)          # z = q without q5 (q2 stays column 2)
    T[5, 2] = 0.5                                 # q5 = 0.5 q2
    return T @ np.linalg.solve(T.T @ H @ T, T.T @ rhs)


def test_stiff_coupling_approaches_the_constrained_dynamics():
    rng = np.random.default_rng(2)
    base = synth.chain_model(1)
    q = rng.uniform(-0.3, 0.3, base["nq"])
    q[5] = 0.5 * q[2]                     # a consistent state: phi = 0, J qd = 0
    qd = rng.uniform(-1, 1, base["nv"])
    qd[5] = 0.5 * qd[2]
    act = rng.uniform(0, 0.5, base["n_mus"])
    u = rng.uniform(0, 1, base["n_mus"])
    want = _nullspace_qdd(_chain_coupled(0, 0), q, qd, act, u)
    errs = []
    for k in (1e6, 1e8, 1e10):
        m = _chain_coupled(k, 0.0)
        _, _, _, st, S = Oracle(m).step(DT, q, qd, act, u, contact=False, stages=True)
        assert st == 0
        errs.append(np.abs(S["qdd"] - want).max() / np.abs(want).max())
    # the penalty solution converges to the constrained one like 1/k
    assert errs[2] < 1e-5 and errs[1] < 1e-3
    assert errs[2] < errs[1] / 30 and errs[1] < errs[0] / 30
    # and the constraint's acceleration vanishes in the limit
    m = _chain_coupled(1e10, 0.0)
    _, _, _, _, S = Oracle(m).step(DT, q, qd, act, u, contact=False, stages=True)
    assert abs(S["qdd"][5] - 0.5 * S["qdd"][2]) < 1e-5 * np.abs(S["qdd"]).max()


@pytest.mark.parametrize("ratio", [0.5, 0.2])
def test_shoulder_rhythm_holds_on_the_whole_body(ratio):
    """The coupled whole body (contact off) keeps each constraint within
    0.05 rad over 200 steps of random excitations (the resisted torque over
    the stiffness), where the uncoupled body drifts at least 3x further."""
    m = synth.shoulder_coupling(synth.human_model(2), scap_ratio=ratio)
    o = Oracle(m)
    q, qd, act = synth.human_initial_state(m, 4)
    # start on the constraint manifold
    for c in range(m["n_eq"]):
        a, b = m["eq_start"][c], m["eq_start"][c + 1]
        dof = m["eq_dof"][a:b]
        q[:, dof[0] + 1] = -m["eq_coef"][a + 1] * q[:, dof[1] + 1]
    u = np.random.default_rng(3).uniform(0, 1, (200, 4, m["n_mus"])).astype(np.float32)
    qo, qdo, ao, st = o.rollout(DT, q.astype(np.float64), qd.astype(np.float64),
                                act.astype(np.float64), u, contact=False, threads=4)
    assert (st == 0).all()
    phi = np.stack([o.coupling(qo[e], qdo[e], DT)[2] for e in range(4)])
    assert np.abs(phi).max() < 0.05
    # uncoupled, the same run drifts further from the rhythm
    mu = dict(m)
    mu["n_eq"] = 0
    ou = Oracle(mu)
    q2, qd2, _, _ = ou.rollout(DT, q.astype(np.float64), qd.astype(np.float64),
                               act.astype(np.float64), u, contact=False, threads=4)
    phi_free = np.stack([o.coupling(q2[e], qd2[e], DT)[2] for e in range(4)])
    assert np.abs(phi_free).max() > 3 * np.abs(phi).max()
