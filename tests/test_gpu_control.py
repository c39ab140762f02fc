"""The control step (ms_controller_step) against the control-step oracle
(oracle/control.py): the observation, the initial sample and the
flow-refined excitations; then, with excitations given, the substeps, the
recorded muscle state, the tracking error and the reward; and the full-size
step (2048 envs, 1024-wide networks, 20 flow steps, 10 substeps) for
determinism and finite rewards.

Tolerances: the observation holds FP32 kinematics (2e-5 m / 2e-5 on rotation
entries) and float32 sinusoids (2e-6 rad); network outputs may differ where
the GPU's and the oracle's inputs round to neighbouring bfloat16 values
(relative 2e-2 of the output scale); the state after n_sub substeps holds n_sub
times the per-step bound 1e-5 (contact off)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import Oracle  # noqa: E402
from oracle import control as ctl  # noqa: E402
from paper_2603_29332_amd import ms, synth  # noqa: E402

DEV = "cuda"
DT = 1e-3


def _t(a, dtype=torch.float32):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


@pytest.fixture(scope="module")
def setup():
    m = synth.human_model(2)
    gm = ms.Model(m)
    keys = np.flatnonzero(m["mass"] > 0)[::2][:10]
    c = ms.Controller(gm, keys, hidden=128, n_sub=2, flow_steps=4, flow_dt=0.25, sigma0=0.2)
    return m, gm, Oracle(m), c, keys


def _state(m, E, seed):
    q, qd, act = synth.human_initial_state(m, E, seed=seed)
    rng = np.random.default_rng(seed)
    qd = (qd + rng.normal(0, 0.2, qd.shape)).astype(np.float32)
    act = rng.uniform(0.05, 0.5, act.shape).astype(np.float32)
    nm = m["n_mus"]
    ms_ = np.stack([rng.uniform(0, 1, (E, nm)), rng.uniform(0, 1, (E, nm)) * m["f0"],
                    rng.uniform(0.8, 1.2, (E, nm)), rng.uniform(-0.5, 0.5, (E, nm))]).astype(np.float32)
    return q, qd, act, ms_


def _oracle_params(p):
    W1, b1, W2, b2, W3, b3 = p
    return [W1.T.copy(), b1, W2.T.copy(), b2, W3.T.copy(), b3]


def test_observation_and_excitations_match_oracle(setup):
    m, gm, o, c, keys = setup
    E, step, t = 6, 7, 0.31
    q, qd, act, mst = _state(m, E, 3)
    tq, tqd, tact, tms = _t(q), _t(qd), _t(act), _t(mst)
    st = torch.zeros(E, dtype=torch.int32, device=DEV)
    rew = torch.zeros(E, device=DEV)
    out = {"obs": torch.zeros(E, c.n_obs, device=DEV), "a0": torch.zeros(E, m["n_mus"], device=DEV),
           "u": torch.zeros(E, m["n_mus"], device=DEV)}
    c.step(tq, tqd, tact, st, tms, step, t, DT, rew, contact=False, out=out)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items()}
    pi, _, log_std = c.params(0)
    fl, wat, _ = c.params(1)
    flow = _oracle_params(fl)
    flow[0] = np.concatenate([flow[0], wat.T], axis=0)   # first layer over [s | a, t]
    pi = _oracle_params(pi)
    nh = len(ctl.hinge_coords(m))
    for e in range(E):
        s = ctl.observation(m, o, q[e], qd[e], mst[:, e], t, e, keys, 52)
        assert s.shape == (c.n_obs,)
        d = np.abs(g["obs"][e] - s)
        k0, r0 = 2 * m["nv"], 2 * m["nv"] + 9 * len(keys) + 4 * m["n_mus"]
        assert d[:k0].max() < 1e-6                                  # q (rotation vector), qd
        assert d[k0:k0 + 9 * len(keys)].max() < 2e-5                # key frames (FP32 kinematics)
        assert d[k0 + 9 * len(keys):r0].max() < 1e-6                # muscle state (F / F0)
        assert d[r0:r0 + nh].max() < 2e-6                           # reference targets
        assert d[r0 + nh:].max() < 2e-5                             # reference key frames
        a0, u = ctl.sample_action(pi, flow, log_std, s, c.n_in, c.n_at, m["n_mus"], e, step, 53,
                                  4, 0.25)
        scale = 1.0 + np.abs(a0).max()
        assert np.abs(g["a0"][e] - a0).max() < 2e-2 * scale, np.abs(g["a0"][e] - a0).max()
        assert np.abs(g["u"][e] - u).max() < 2e-2 * scale, np.abs(g["u"][e] - u).max()
    # the flow moved the sample and the clamp bit
    assert np.abs(g["u"] - np.clip(g["a0"], 0, 1)).max() > 1e-3
    assert (g["u"] == 0).any() and (g["u"] > 0).any()


def test_substeps_muscle_state_and_reward_match_oracle(setup):
    m, gm, o, c, keys = setup
    E, t = 5, 0.5
    q, qd, act, mst = _state(m, E, 4)
    u = np.random.default_rng(8).uniform(0, 1, (E, m["n_mus"])).astype(np.float32)
    tq, tqd, tact, tms = _t(q), _t(qd), _t(act), _t(mst)
    st = torch.zeros(E, dtype=torch.int32, device=DEV)
    napp = torch.zeros(E, dtype=torch.int32, device=DEV)
    rew = torch.zeros(E, device=DEV)
    delta = torch.zeros(E, len(ctl.hinge_coords(m)) + 3 * len(keys), device=DEV)
    c.step(tq, tqd, tact, st, tms, 0, t, DT, rew, contact=False, u_in=_t(u),
           out={"delta": delta, "n_applied": napp})
    torch.cuda.synchronize()
    gq, gqd, gact, gms, gr, gd = (x.cpu().numpy() for x in (tq, tqd, tact, tms, rew, delta))
    assert (st.cpu().numpy() == 0).all() and (napp.cpu().numpy() == 2).all()
    disc = _oracle_params(c.params(2)[0])
    f0max = float(m["f0"].max())
    for e in range(E):
        qo, qdo, ao, sto, last = ctl.substeps(o, DT, q[e], qd[e], act[e], u[e], 2, False)
        assert sto == 0
        for a, b in zip((gq[e], gqd[e], gact[e]), (qo, qdo, ao)):
            assert np.abs(a - b).max() / max(np.abs(b).max(), 1.0) <= 2e-5
        assert np.abs(gms[0, e] - last[0]).max() < 1e-6
        assert np.abs(gms[1, e] - last[1]).max() < 2e-4 * f0max
        assert np.abs(gms[2, e] - last[2]).max() < 1e-4 * (1 + np.abs(last[2]).max())
        assert np.abs(gms[3, e] - last[3]).max() < 1e-4 * (1 + np.abs(last[3]).max())
        dl = ctl.tracking_error(m, o, qo, e, t + 2 * DT, keys, 52)
        assert np.abs(gd[e] - dl).max() < 1e-4
        r = ctl.reward(disc, dl, c.n_din)
        assert abs(gr[e] - r) < 2e-2 * max(r, 0.1), (gr[e], r)


def test_full_size_control_steps_are_deterministic():
    """2048 envs, the paper's network sizes (1024 wide), 20 flow steps of
    0.05, 10 substeps per control step: three control steps twice give the
    same bits, finite rewards and states."""
    m = synth.human_model(2)
    gm = ms.Model(m)
    keys = np.flatnonzero(m["mass"] > 0)[::2][:10]
    c = ms.Controller(gm, keys)
    E = 2048
    runs = []
    for _ in range(2):
        q, qd, act = synth.human_initial_state(m, E)
        tq, tqd, tact = _t(q), _t(qd), _t(act)
        tms = torch.zeros(4, E, m["n_mus"], device=DEV)
        st = torch.zeros(E, dtype=torch.int32, device=DEV)
        rew = torch.zeros(3, E, device=DEV)
        for k in range(3):
            c.step(tq, tqd, tact, st, tms, k, k * 10 * DT, DT, rew[k], contact=True)
        torch.cuda.synchronize()
        runs.append([x.cpu().numpy() for x in (tq, tqd, tact, tms, st, rew)])
    a, b = runs
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    ok = a[4] == 0
    assert ok.mean() > 0.95
    assert np.isfinite(a[5][:, ok]).all() and (a[5][:, ok] > 0).all()
    assert np.isfinite(a[0][ok]).all()
