"""Uneven batches through the C ABI: three models of different sizes stepped
in one call (per-model kernels on forked streams, replayed as a HIP graph).
Every configuration must give, bit for bit, what ms_rollout gives for each
model alone; that path is itself held to the FP64 oracle by the parity
tests."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2603_29332_amd import ms, synth  # noqa: E402

DEV = "cuda"
DT = 1e-3


def _t(a, dtype=torch.float32):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


@pytest.fixture(scope="module")
def three():
    ms_ = [synth.chain_model(31), synth.human_model(32, full=False), synth.human_model(33)]
    inits = [synth.chain_initial_state, synth.human_initial_state, synth.human_initial_state]
    n_env = [64, 96, 128]                       # ragged against 2- and 4-env workgroups
    return ms_, [ms.Model(m) for m in ms_], inits, n_env


def _fresh(m, init, n):
    q, qd, act = init(m, n)
    return [_t(q), _t(qd), _t(act), torch.zeros(n, dtype=torch.int32, device=DEV),
            torch.zeros(n, m["n_mus"], device=DEV)]


def _exc(x, step0):
    rho, s, mean, _ = synth.ar1_constants(DT)
    return dict(kind=ms.EXC_AR1, seed=34, step0=step0, x=x, ar1=(rho, s, mean))


def _alone(mods, gms, inits, n_env, T, calls=1):
    out = []
    for m, gm, init, n in zip(mods, gms, inits, n_env):
        q, qd, act, st, x = _fresh(m, init, n)
        for c in range(calls):
            gm.rollout(q, qd, act, st, T, DT, True, **_exc(x, c * T))
        torch.cuda.synchronize()
        out.append([v.cpu().numpy() for v in (q, qd, act, st, x)])
    return out


def _batched(mods, b, inits, n_env, T, calls=1, contact=True):
    bufs = [_fresh(m, init, n) for m, init, n in zip(mods, inits, n_env)]
    for c in range(calls):
        b.rollout([tuple(v[:4]) for v in bufs], [_exc(v[4], c * T) for v in bufs], T, DT,
                  contact=contact)
    torch.cuda.synchronize()
    return [[v.cpu().numpy() for v in bb] for bb in bufs]


def _same(a, b):
    for x, y in zip(a, b):
        for u, v in zip(x, y):
            assert np.array_equal(u, v)


def test_batch_matches_each_model_alone_in_every_configuration(three):
    mods, gms, inits, n_env = three
    T = 20
    ref = _alone(mods, gms, inits, n_env, T)
    b = ms.Batch(gms, n_env)
    for cfg, mode in (([1, 1, 1], ms.ISSUE_CONCURRENT), ([2, 4, 1], ms.ISSUE_CONCURRENT_MOST_WORK),
                      ([4, 2, 4], ms.ISSUE_SERIAL), ([2, 2, 4], ms.ISSUE_CONCURRENT)):
        b.set_config(cfg, mode)
        assert b.config() == (cfg, mode)
        _same(_batched(mods, b, inits, n_env, T), ref)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_graph_replay_continues_the_rollout(three, mode):
    mods, gms, inits, n_env = three
    T = 10
    ref = _alone(mods, gms, inits, n_env, T, calls=3)
    b = ms.Batch(gms, n_env)
    b.set_config([0, 4, 2], mode)
    _same(_batched(mods, b, inits, n_env, T, calls=3), ref)


def test_autotune_picks_a_valid_configuration_and_leaves_states(three):
    mods, gms, inits, n_env = three
    b = ms.Batch(gms, n_env)
    bufs = [_fresh(m, init, n) for m, init, n in zip(mods, inits, n_env)]
    before = [[v.cpu().numpy().copy() for v in bb] for bb in bufs]
    w, lf = b.autotune([tuple(v[:4]) for v in bufs], [_exc(v[4], 0) for v in bufs], 5, DT)
    torch.cuda.synchronize()
    assert all(x in (1, 2, 4) for x in w) and lf in (0, 1, 2)
    after = [[v.cpu().numpy() for v in bb] for bb in bufs]
    _same(after, before)
    # and the tuned batch still matches the models alone
    _same(_batched(mods, b, inits, n_env, 10), _alone(mods, gms, inits, n_env, 10))


def test_oversized_workgroup_is_rejected(three):
    mods, gms, inits, n_env = three
    b = ms.Batch([gms[2]], [8])
    if gms[2].info["lds_shared_bytes"] + gms[2].info["lds_bytes"] * 4 > 160 * 1024:
        with pytest.raises(ms.MsError):
            b.set_config([4], 0)
    else:
        b.set_config([4], 0)


def test_full_size_batch_matches_each_model_alone(three):
    """The uneven-batch workload at its full size (4096 + 4096 + 8192 envs of
    the three models, autotuned, replayed as a graph) equals each model's
    rollout alone, bit for bit."""
    mods, gms, inits, _ = three
    n_env = [4096, 4096, 8192]
    T = 20
    b = ms.Batch(gms, n_env)
    bufs = [_fresh(m, init, n) for m, init, n in zip(mods, inits, n_env)]
    b.autotune([tuple(v[:4]) for v in bufs], [_exc(v[4], 0) for v in bufs], T, DT)
    _same(_batched(mods, b, inits, n_env, T), _alone(mods, gms, inits, n_env, T))


def test_calls_recorded_in_a_caller_graph_replay_like_eager_calls(three):
    """ms_rollout and ms_batch_rollout (concurrent issue: its forked streams
    join the caller's capture) recorded inside a caller's stream capture (a
    torch CUDA graph): each of three replays, with eager calls and
    synchronisations between them, advances the state exactly as the same
    calls made eagerly."""
    mods, gms, inits, n_env = three
    T = 5
    m, gm, init, n = mods[2], gms[2], inits[2], n_env[2]
    A, B = _fresh(m, init, n), _fresh(m, init, n)
    kw = dict(kind=ms.EXC_IID, seed=3, step0=7)
    gm.reserve(n)        # no allocation may happen inside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        gm.rollout(*A[:4], T, DT, True, **kw)
    b = ms.Batch(gms, n_env)
    b.set_config([2, 4, 4], ms.ISSUE_CONCURRENT)
    bA = [_fresh(mm, ii, nn) for mm, ii, nn in zip(mods, inits, n_env)]
    bB = [_fresh(mm, ii, nn) for mm, ii, nn in zip(mods, inits, n_env)]
    g2 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g2):
        b.rollout([tuple(v[:4]) for v in bA], [_exc(v[4], 0) for v in bA], T, DT)
    for _ in range(3):
        g.replay()
        gm.rollout(*B[:4], T, DT, True, **kw)
        g2.replay()
        b.rollout([tuple(v[:4]) for v in bB], [_exc(v[4], 0) for v in bB], T, DT)
        torch.cuda.synchronize()
        for x, y in zip(A[:4], B[:4]):
            assert torch.equal(x, y)
        for u, v in zip(bA, bB):
            for x, y in zip(u, v):
                assert torch.equal(x, y)
