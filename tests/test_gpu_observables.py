"""Per-step observables of ms_rollout_record against the FP64 oracle: the
activation driving each step's force, the Hill force, normalised fibre
length and velocity, the power |F Ldot| and the world frames of key nodes,
teacher-forced (each recorded step starts from the GPU state read back
before it), on both step schedules; records of a longer call every k steps;
and the applied-step counters."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import Oracle  # noqa: E402
from paper_2603_29332_amd import ms, synth  # noqa: E402

DEV = "cuda"
KEYS = ("act", "force", "lm", "vm", "power", "xpos", "xmat")


def _t(a, dtype=torch.float32):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def _setup(which, schedule):
    if which == "chain":
        m = synth.chain_model(1)
        init, dt, contact = synth.chain_initial_state, 2e-3, False
        keys = np.arange(m["n_node"])
    else:
        m = synth.human_model(2)
        init, dt, contact = synth.human_initial_state, 1e-3, True
        keys = np.flatnonzero(m["mass"] > 0)[::2][:10]     # ten key bodies
    gm = ms.Model(m)
    gm.set_schedule(schedule)
    gm.set_key_nodes(keys)
    return m, gm, Oracle(m), init, dt, contact, keys


def _obs_buffers(m, E, n_rec, n_key):
    nm = m["n_mus"]
    shapes = dict(act=(n_rec, E, nm), force=(n_rec, E, nm), lm=(n_rec, E, nm),
                  vm=(n_rec, E, nm), power=(n_rec, E, nm), xpos=(n_rec, E, n_key, 3),
                  xmat=(n_rec, E, n_key, 9))
    return {k: torch.full(s, float("nan"), device=DEV) for k, s in shapes.items()}


@pytest.mark.parametrize("schedule", [ms.SCHED_FUSED, ms.SCHED_SPLIT])
@pytest.mark.parametrize("which", ["chain", "human"])
def test_observables_match_oracle_teacher_forced(which, schedule):
    m, gm, o, init, dt, contact, keys = _setup(which, schedule)
    E, T = 8, 3
    q, qd, act = init(m, E)
    rng = np.random.default_rng(17)
    qd = (qd + rng.normal(0, 0.3, qd.shape)).astype(np.float32)
    act = rng.uniform(0.05, 0.6, act.shape).astype(np.float32)
    tq, tqd, tact = _t(q), _t(qd), _t(act)
    st = torch.zeros(E, dtype=torch.int32, device=DEV)
    napp = torch.zeros(E, dtype=torch.int32, device=DEV)
    f0max = float(m["f0"].max())
    for t in range(T):
        qs, qds, acts = (x.cpu().numpy() for x in (tq, tqd, tact))
        u = synth.excitation_iid(30 + t, E, m["n_mus"], 0)
        obs = _obs_buffers(m, E, 1, len(keys))
        gm.rollout_record(tq, tqd, tact, st, 1, dt, contact, kind=ms.EXC_ARRAY, u=_t(u[None]),
                          every=1, obs=obs, n_applied=napp)
        torch.cuda.synchronize()
        g = {k: v.cpu().numpy()[0] for k, v in obs.items()}
        for e in range(E):
            _, _, _, sto, S = o.step(dt, qs[e], qds[e], acts[e], u[e], contact=contact,
                                     stages=True)
            assert sto == 0
            assert np.abs(g["act"][e] - S["act"]).max() < 2e-7
            assert np.abs(g["force"][e] - S["F"]).max() < 2e-4 * f0max
            assert np.abs(g["lm"][e] - S["lm"]).max() < 1e-4 * (1 + np.abs(S["lm"]).max())
            assert np.abs(g["vm"][e] - S["vm"]).max() < 1e-4 * (1 + np.abs(S["vm"]).max())
            pw = np.abs(S["F"] * S["Ldot"])
            ptol = 2e-4 * f0max * np.abs(S["Ldot"]) + np.abs(S["F"]) * 1e-5 * (
                1 + np.abs(S["Ldot"]).max()) + 1e-6
            assert (np.abs(g["power"][e] - pw) <= ptol).all()
            R, p = o.fk(qs[e].astype(np.float64))
            assert np.abs(g["xpos"][e] - p[keys]).max() < 2e-5
            assert np.abs(g["xmat"][e] - R[keys].reshape(len(keys), 9)).max() < 2e-5
    assert (st.cpu().numpy() == 0).all()
    assert (napp.cpu().numpy() == T).all()


@pytest.mark.parametrize("schedule", [ms.SCHED_FUSED, ms.SCHED_SPLIT])
def test_records_every_k_steps_and_state_unchanged(schedule):
    """One call of 7 steps recording every 3rd step (steps 0, 3, 6) equals
    the same call recording every step, at those steps, bit for bit; the
    state ends as a plain ms_rollout's; a frozen env's counter stays 0."""
    m, gm, o, init, dt, contact, keys = _setup("human", schedule)
    E, T = 12, 7
    q, qd, act = init(m, E)
    q[5, 20] = np.nan
    kw = dict(kind=ms.EXC_AR1, seed=9, step0=4, ar1=synth.ar1_constants(dt)[:3])
    runs = []
    for every in (1, 3, None):
        tq, tqd, tact = _t(q), _t(qd), _t(act)
        st = torch.zeros(E, dtype=torch.int32, device=DEV)
        x = torch.zeros(E, m["n_mus"], device=DEV)
        napp = torch.zeros(E, dtype=torch.int32, device=DEV)
        if every is None:
            gm.rollout(tq, tqd, tact, st, T, dt, contact, x=x, **kw)
            obs = {}
        else:
            obs = _obs_buffers(m, E, -(-T // every), len(keys))
            gm.rollout_record(tq, tqd, tact, st, T, dt, contact, x=x, every=every, obs=obs,
                              n_applied=napp, **kw)
        torch.cuda.synchronize()
        runs.append(([v.cpu().numpy() for v in (tq, tqd, tact, st, x)],
                     {k: v.cpu().numpy() for k, v in obs.items()}, napp.cpu().numpy()))
    (s1, o1, n1), (s3, o3, n3), (s0, _, _) = runs
    for a, b, c in zip(s1, s3, s0):
        assert np.array_equal(a, b, equal_nan=True) and np.array_equal(a, c, equal_nan=True)
    for k in KEYS:
        assert o3[k].shape[0] == 3
        ok = np.arange(E) != 5
        assert np.array_equal(o1[k][[0, 3, 6]][:, ok], o3[k][:, ok]), k
        assert np.isnan(o3[k][:, 5]).all(), k          # skipped steps leave entries unwritten
    assert list(n1) == [T if e != 5 else 0 for e in range(E)] and list(n3) == list(n1)


def test_record_arguments_are_checked():
    m, gm, o, init, dt, contact, keys = _setup("chain", ms.SCHED_AUTO)
    E = 4
    q, qd, act = (_t(x) for x in init(m, E))
    st = torch.zeros(E, dtype=torch.int32, device=DEV)
    obs = _obs_buffers(m, E, 1, len(keys))
    with pytest.raises(ms.MsError):
        gm.rollout_record(q, qd, act, st, 1, dt, False, kind=ms.EXC_IID, every=0, obs=obs)
    gm.set_key_nodes([])
    with pytest.raises(ms.MsError):
        gm.rollout_record(q, qd, act, st, 1, dt, False, kind=ms.EXC_IID, every=1,
                          obs={"xpos": obs["xpos"]})
    with pytest.raises(ms.MsError):
        gm.set_key_nodes([m["n_node"]])
