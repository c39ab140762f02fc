"""Policy-driven rollouts on the GPU: observations and excitations against
the oracle's definitions, and the rollout against the plain step driven by
the same excitations."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_2603_29332_amd import ms, synth  # noqa: E402

DEV = "cuda"
DT = 1e-3


def _t(a, dtype=torch.float32):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


@pytest.fixture(scope="module")
def setup():
    m = synth.human_model(2)
    gm = ms.Model(m)
    p = ms.Policy(gm, hidden=512, n_ref=140, ref_seed=52, seed=51)
    return m, gm, p, oracle.Oracle(m)


def _states(m, o, E):
    """Seeded whole-body states after 40 oracle steps (non-zero velocities)."""
    q, qd, act = synth.human_initial_state(m, E, seed=17)
    u, _ = synth.excitation_sequence("ar1", 5, E, m["n_mus"], 40, DT)
    q, qd, act, st = o.rollout(DT, q, qd, act, u, contact=True)
    assert (st == 0).all()
    return q.astype(np.float32), qd.astype(np.float32), act.astype(np.float32)


def test_observation_and_excitations_match_oracle(setup):
    m, gm, p, o = setup
    assert (p.n_obs, p.n_in, p.n_out) == (300, 304, 700)
    E, env0, t = 136, 1000, 0.123
    q, qd, _ = _states(m, o, E)
    u = torch.zeros(E, m["n_mus"], device=DEV)
    obs = torch.zeros(E, p.n_obs, device=DEV)
    p.act(_t(q), _t(qd), t, u, env0=env0, obs=obs)
    torch.cuda.synchronize()
    amp, freq, phase = synth.reference_params(52, E, 140, envs=np.arange(env0, env0 + E))
    obs_o = oracle.policy_obs(m, q, qd, t, amp, freq, phase)
    og = obs.cpu().numpy()
    assert np.abs(og - obs_o).max() <= 2e-6 * max(1.0, np.abs(obs_o).max())
    W1, b1, W2, b2, W3, b3 = p.params()
    uo = oracle.policy_act([W1.T.copy(), b1, W2.T.copy(), b2, W3.T.copy(), b3], obs_o, p.n_in)
    ug = u.cpu().numpy()
    assert ((ug >= 0) & (ug <= 1)).all()
    # bfloat16 operands (rounding points mirrored by the oracle), float32 sums
    assert np.abs(ug - uo).max() < 2e-3


def test_policy_rollout_equals_steps_driven_by_its_recorded_excitations(setup):
    m, gm, p, o = setup
    E, T, decim = 64, 10, 2
    q, qd, act = _states(m, o, E)
    tq, tqd, tact = _t(q), _t(qd), _t(act)
    st = torch.zeros(E, dtype=torch.int32, device=DEV)
    rec = torch.zeros(T // decim, E, m["n_mus"], device=DEV)
    p.rollout(tq, tqd, tact, st, T, decim, DT, contact=True, t0=0.5, u_record=rec)
    # the first decision equals the policy evaluated at the initial state
    u0 = torch.zeros(E, m["n_mus"], device=DEV)
    p.act(_t(q), _t(qd), 0.5, u0)
    torch.cuda.synchronize()
    assert np.array_equal(rec[0].cpu().numpy(), u0.cpu().numpy())
    # the same run as plain array-driven steps
    useq = rec.repeat_interleave(decim, dim=0).contiguous()
    eq, eqd, eact = _t(q), _t(qd), _t(act)
    est = torch.zeros(E, dtype=torch.int32, device=DEV)
    gm.rollout(eq, eqd, eact, est, T, DT, True, kind=ms.EXC_ARRAY, u=useq)
    torch.cuda.synchronize()
    for a, b in ((tq, eq), (tqd, eqd), (tact, eact), (st, est)):
        assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())


def test_full_size_policy_rollout_sampled_against_oracle(setup):
    """The policy-driven workload at its full size: 65,536 envs, decisions
    every 2 steps, the surrogate geometry with per-env fallback. An untrained
    network fails the residual check everywhere, so every env-step takes the
    exact geometry; 16 sampled envs are compared with the oracle driven by
    the recorded excitations."""
    m, gm, p, o = setup
    E, T, decim = 65536, 10, 2
    q, qd, act = synth.human_initial_state(m, E)
    tq, tqd, tact = _t(q), _t(qd), _t(act)
    st = torch.zeros(E, dtype=torch.int32, device=DEV)
    fb = torch.zeros(E, dtype=torch.int32, device=DEV)
    rec = torch.zeros(T // decim, E, m["n_mus"], device=DEV)
    sg = ms.Surrogate(gm, hidden=512, seed=41)
    p.rollout(tq, tqd, tact, st, T, decim, DT, contact=True, t0=0.0, surrogate=sg, tol=1e-4,
              fb_count=fb, u_record=rec)
    torch.cuda.synchronize()
    assert (fb.cpu().numpy() == T).all()
    assert ((st.cpu().numpy() & ~ms.MS_ST_FALLBACK) == 0).all()
    sub = np.arange(17, E, 4096)
    u = np.repeat(rec.cpu().numpy()[:, sub], decim, axis=0)
    qo, qdo, ao, so = o.rollout(DT, q[sub], qd[sub], act[sub], u, contact=True)
    assert (so == 0).all()
    qg, qdg, ag = (v.cpu().numpy()[sub] for v in (tq, tqd, tact))
    assert np.abs(qg[:, 7:] - qo[:, 7:]).max() < 1e-5
    assert np.abs(qdg - qdo).max() < 1e-4 * max(np.abs(qdo).max(), 1.0)
    assert np.abs(ag - ao).max() < 1e-6
