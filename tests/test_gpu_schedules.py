"""The split step schedule (three kernels per physics step exchanging
per-env intermediates through a device workspace) against the fused one
(one kernel per rollout): both perform the same operations in the same
order, so every result must agree bit for bit — states, activations,
smooth-noise states, status words and fallback counts — for every model,
excitation source, failure path, the surrogate step and policy-driven
rollouts. Parity of the fused step with the FP64 oracle is covered in
test_gpu_parity.py; the models that run split by default (the whole body)
also run split there."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2603_29332_amd import ms, synth  # noqa: E402

DEV = "cuda"
DT = 1e-3


def _t(a, dtype=torch.float32):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


MODELS = {
    "chain": (lambda: synth.chain_model(1), synth.chain_initial_state),
    "human40": (lambda: synth.human_model(32, full=False), synth.human_initial_state),
    "human": (lambda: synth.human_model(2), synth.human_initial_state),
}


@pytest.fixture(scope="module")
def built():
    out = {}
    for k, (mk, init) in MODELS.items():
        m = mk()
        fused, split = ms.Model(m), ms.Model(m)
        fused.set_schedule(ms.SCHED_FUSED)
        split.set_schedule(ms.SCHED_SPLIT)
        out[k] = (m, init, fused, split)
    return out


def _state(m, init, E, seed):
    q, qd, act = init(m, E)
    rng = np.random.default_rng(seed)
    qd = (qd + rng.normal(0, 0.2, qd.shape)).astype(np.float32)
    act = rng.uniform(0.0, 0.5, act.shape).astype(np.float32)
    return q, qd, act


def _run(gm, m, q, qd, act, T, contact, kind, seed=12, u=None, step0=0, x0=None):
    E = q.shape[0]
    tq, tqd, tact = _t(q), _t(qd), _t(act)
    st = torch.zeros(E, dtype=torch.int32, device=DEV)
    x = _t(x0 if x0 is not None else np.zeros((E, m["n_mus"]), np.float32))
    kw = dict(kind=kind, seed=seed, step0=step0)
    if kind == ms.EXC_ARRAY:
        kw["u"] = _t(u)
    if kind == ms.EXC_AR1:
        kw["x"] = x
        kw["ar1"] = synth.ar1_constants(DT)[:3]
    gm.rollout(tq, tqd, tact, st, T, DT, contact, **kw)
    torch.cuda.synchronize()
    return [v.cpu().numpy() for v in (tq, tqd, tact, st, x)]


def _same(a, b):
    for k, (x, y) in enumerate(zip(a, b)):
        assert np.array_equal(x, y, equal_nan=True), (k, np.nanmax(np.abs(x.astype(np.float64) -
                                                                          y.astype(np.float64))))


def test_default_schedules(built):
    for k, (m, init, _, _) in built.items():
        gm = ms.Model(m)
        want = ms.SCHED_SPLIT if k == "human" else ms.SCHED_FUSED
        assert gm.schedule() == want, k


@pytest.mark.parametrize("name", list(MODELS))
@pytest.mark.parametrize("kind", [ms.EXC_AR1, ms.EXC_IID, ms.EXC_ARRAY])
def test_split_equals_fused(built, name, kind):
    m, init, fused, split = built[name]
    E, T = 93, 15                  # several workgroups of every kernel and a ragged tail
    q, qd, act = _state(m, init, E, 3)
    u = None
    if kind == ms.EXC_ARRAY:
        u = np.random.default_rng(4).uniform(-0.1, 1.1, (T, E, m["n_mus"])).astype(np.float32)
    x0 = np.random.default_rng(5).normal(0, 0.1, (E, m["n_mus"])).astype(np.float32)
    a = _run(fused, m, q, qd, act, T, True, kind, u=u, step0=11, x0=x0)
    b = _run(split, m, q, qd, act, T, True, kind, u=u, step0=11, x0=x0)
    assert np.isfinite(a[0]).all()
    _same(a, b)
    # and the states moved
    assert np.abs(a[1] - qd).max() > 1e-3


def test_split_step_batch_equals_fused(built):
    m, init, fused, split = built["human"]
    E = 70
    q, qd, act = _state(m, init, E, 6)
    u = np.random.default_rng(7).uniform(0, 1, (3, E, m["n_mus"])).astype(np.float32)
    outs = []
    for gm in (fused, split):
        tq, tqd, tact = _t(q), _t(qd), _t(act)
        st = torch.zeros(E, dtype=torch.int32, device=DEV)
        for k in range(3):
            gm.step_batch(tq, tqd, tact, st, _t(u[k]), DT, True)
        torch.cuda.synchronize()
        outs.append([v.cpu().numpy() for v in (tq, tqd, tact, st)])
    _same(*outs)


def test_split_failure_paths_equal_fused(built):
    """Non-finite positions, velocities and activations: flagged and frozen
    alike by both schedules (the smooth-noise state still advances)."""
    m, init, fused, split = built["human"]
    E, T = 20, 4
    q, qd, act = _state(m, init, E, 8)
    q[1, 9] = np.nan
    qd[4, 30] = np.inf
    act[6, 100] = np.nan
    x0 = np.zeros((E, m["n_mus"]), np.float32)
    a = _run(fused, m, q, qd, act, T, True, ms.EXC_AR1, x0=x0)
    b = _run(split, m, q, qd, act, T, True, ms.EXC_AR1, x0=x0)
    _same(a, b)
    assert list(np.flatnonzero(a[3])) == [1, 4, 6]
    assert (a[3][[1, 4, 6]] == ms.MS_ST_NONFINITE).all()
    assert np.array_equal(a[0][1], q[1], equal_nan=True)
    assert np.array_equal(a[2][6], act[6], equal_nan=True)
    assert np.abs(a[4][1]).max() > 0        # noise state advanced on a frozen env


def test_split_nonspd_equals_fused():
    """A massless, undamped leaf hinge on the whole body makes M singular for
    every env: both schedules flag it and keep the state."""
    m = dict(synth.human_model(2))
    for k in ("mass", "inertia", "com", "damping"):
        m[k] = m[k].copy()
    leaf = [i for i in range(m["n_node"]) if i not in set(m["parent"])][0]
    m["mass"][leaf] = 0.0
    m["inertia"][leaf] = 0.0
    dof = 6 + leaf - 1
    m["damping"][dof] = 0.0
    # no muscle or contact may act on the massless link (their implicit
    # damping would make its pivot positive)
    keep = [i for i in range(m["n_mus"])
            if leaf not in m["via_node"][m["via_start"][i]:m["via_start"][i + 1]]]
    vs, vn, vp = [0], [], []
    for i in keep:
        a, b = m["via_start"][i], m["via_start"][i + 1]
        vn += list(m["via_node"][a:b])
        vp += list(m["via_pos"][a:b])
        vs.append(len(vn))
    for k in ("f0", "l_opt", "l_slack", "v_max", "tau_act", "tau_deact"):
        m[k] = m[k][keep]
    m["via_start"], m["via_node"], m["via_pos"] = vs, vn, np.array(vp)
    cs = [c for c in range(m["n_con"]) if m["con_node"][c] != leaf]
    m["con_node"], m["con_pos"], m["con_radius"] = (m["con_node"][cs], m["con_pos"][cs],
                                                     m["con_radius"][cs])
    m = synth._finish(m)
    fused, split = ms.Model(m), ms.Model(m)
    fused.set_schedule(ms.SCHED_FUSED)
    split.set_schedule(ms.SCHED_SPLIT)
    E = 9
    q, qd, act = synth.human_initial_state(m, E)
    u = np.zeros((2, E, m["n_mus"]), np.float32)
    a = _run(fused, m, q, qd, act, 2, True, ms.EXC_ARRAY, u=u)
    b = _run(split, m, q, qd, act, 2, True, ms.EXC_ARRAY, u=u)
    _same(a, b)
    assert (a[3] == ms.MS_ST_NONSPD).all()
    assert np.array_equal(a[0], q)


def test_split_surrogate_equals_fused(built):
    """The surrogate step on both schedules: a network whose output layer is
    zero returns its shift, the geometry at a reference pose; envs near it
    take the prediction at a 1 mm check, the others fall back."""
    m, init, fused, split = built["human"]
    E, T = 64, 3
    q, qd, act = _state(m, init, E, 9)
    far = np.arange(E) % 3 == 0
    rng = np.random.default_rng(13)
    near = ~far
    q[near] = q[1]
    q[near, 7:] += rng.uniform(-1e-6, 1e-6, (near.sum(), m["nq"] - 7)).astype(np.float32)
    q[far, 7:] += 0.3
    outs = []
    for gm in (fused, split):
        s = ms.Surrogate(gm, hidden=64, seed=3)
        ps = s.params()
        ps[4][:] = 0.0
        ps[5][:] = 0.0
        s.set_params(ps)
        L = torch.zeros(1, m["n_mus"], device=DEV)
        r = torch.zeros(1, m["n_mus"], 3, device=DEV)
        # the shift: the exact geometry at env 1's pose (a near env)
        gm.geometry(_t(q[1:2]), L, r)
        torch.cuda.synchronize()
        y = np.concatenate([L.cpu().numpy()[0], r.cpu().numpy()[0].reshape(-1)]) + 2e-4
        s.set_norm(y.astype(np.float32), np.ones(s.n_out, np.float32))
        tq, tqd, tact = _t(q), _t(qd), _t(act)
        st = torch.zeros(E, dtype=torch.int32, device=DEV)
        fb = torch.zeros(E, dtype=torch.int32, device=DEV)
        x = torch.zeros(E, m["n_mus"], device=DEV)
        gm.rollout_surrogate(s, tq, tqd, tact, st, T, DT, True, tol=1e-3, fb_count=fb,
                             kind=ms.EXC_AR1, seed=5, x=x, ar1=synth.ar1_constants(DT)[:3])
        torch.cuda.synchronize()
        outs.append([v.cpu().numpy() for v in (tq, tqd, tact, st, x, fb)])
    _same(*outs)
    fb = outs[0][5]
    assert fb[far].min() == T and fb[~far].max() < T     # both branches exercised


def test_split_policy_rollout_equals_fused(built):
    m, init, fused, split = built["human"]
    E, T = 40, 6
    q, qd, act = _state(m, init, E, 10)
    outs = []
    for gm in (fused, split):
        pol = ms.Policy(gm, hidden=128, n_ref=140, ref_seed=52, seed=51)
        tq, tqd, tact = _t(q), _t(qd), _t(act)
        st = torch.zeros(E, dtype=torch.int32, device=DEV)
        pol.rollout(tq, tqd, tact, st, T, 2, DT, contact=True)
        torch.cuda.synchronize()
        outs.append([v.cpu().numpy() for v in (tq, tqd, tact, st)])
    _same(*outs)


def test_split_workspace_grows_and_is_reserved_before_capture(built):
    """A larger batch after a smaller one grows the workspace; inside a stream
    capture a growth is refused before anything is launched, and after
    ms_model_reserve the captured rollout replays like eager calls."""
    m, init, fused, _ = built["human"]
    gm = ms.Model(m)
    assert gm.schedule() == ms.SCHED_SPLIT
    for E in (17, 150):
        q, qd, act = _state(m, init, E, 11)
        a = _run(fused, m, q, qd, act, 3, True, ms.EXC_IID)
        b = _run(gm, m, q, qd, act, 3, True, ms.EXC_IID)
        _same(a, b)
    E = 300
    q, qd, act = _state(m, init, E, 12)
    tq, tqd, tact = _t(q), _t(qd), _t(act)
    st = torch.zeros(E, dtype=torch.int32, device=DEV)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with pytest.raises(ms.MsError) as e:
        with torch.cuda.graph(g):
            gm.rollout(tq, tqd, tact, st, 2, DT, True, kind=ms.EXC_IID, seed=1)
    assert e.value.code == -1
    gm.reserve(E)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        gm.rollout(tq, tqd, tact, st, 2, DT, True, kind=ms.EXC_IID, seed=1)
    ref = [_t(q), _t(qd), _t(act), torch.zeros(E, dtype=torch.int32, device=DEV)]
    for _ in range(2):
        g.replay()
        fused.rollout(*ref, 2, DT, True, kind=ms.EXC_IID, seed=1)
        torch.cuda.synchronize()
        for x, y in zip((tq, tqd, tact, st), ref):
            assert torch.equal(x, y)


@pytest.mark.parametrize("E,parts", [(1, 2), (93, 2), (93, 3), (5, 4), (4097, 2), (4097, 4)])
def test_stream_parts_equal_one_stream(built, E, parts):
    """The split step over concurrent parts of the batch, each on a stream of
    its own (forced for every batch size, including more parts than envs, and
    the automatic choice at 4097 envs), gives the bits of the one-stream
    split step and of the fused step, also when captured into a graph after
    ms_model_reserve and replayed."""
    m, init, fused, _ = built["human"]
    one, two, auto = ms.Model(m), ms.Model(m), ms.Model(m)
    one.set_split_streams(1)
    two.set_split_streams(parts)
    q, qd, act = _state(m, init, E, 14)
    x0 = np.random.default_rng(15).normal(0, 0.1, (E, m["n_mus"])).astype(np.float32)
    ref = _run(one, m, q, qd, act, 4, True, ms.EXC_AR1, x0=x0)
    _same(ref, _run(two, m, q, qd, act, 4, True, ms.EXC_AR1, x0=x0))
    _same(ref, _run(auto, m, q, qd, act, 4, True, ms.EXC_AR1, x0=x0))
    if E <= 93:
        _same(ref, _run(fused, m, q, qd, act, 4, True, ms.EXC_AR1, x0=x0))
    gm = ms.Model(m)
    gm.set_split_streams(parts)
    gm.reserve(E)
    tq, tqd, tact = _t(q), _t(qd), _t(act)
    st = torch.zeros(E, dtype=torch.int32, device=DEV)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        gm.rollout(tq, tqd, tact, st, 2, DT, True, kind=ms.EXC_IID, seed=1)
    want = [_t(q), _t(qd), _t(act), torch.zeros(E, dtype=torch.int32, device=DEV)]
    for _ in range(3):
        g.replay()
        one.rollout(*want, 2, DT, True, kind=ms.EXC_IID, seed=1)
        torch.cuda.synchronize()
        for x, y in zip((tq, tqd, tact, st), want):
            assert torch.equal(x, y)


def test_stream_parts_argument_bounds(built):
    m = built["human"][0]
    gm = ms.Model(m)
    for bad in (-1, 5):
        with pytest.raises(ms.MsError):
            gm.set_split_streams(bad)
    for ok in (0, 1, 4):
        gm.set_split_streams(ok)


def test_split_parts_cover_the_batch(built):
    """ms_model_split_parts: contiguous non-empty parts that cover the batch,
    as many as asked for at these sizes (fewer only when some part would be
    empty); with two parts the first is at least half the batch; one part
    on the fused schedule."""
    m = built["human"][0]
    gm = ms.Model(m)
    for streams in (0, 1, 2, 3, 4):
        gm.set_split_streams(streams)
        for n in (1, 3, 93, 2048, 4096, 4097, 8192):
            b = gm.split_parts(n)
            want = streams if streams else (2 if n >= 4096 else 1)
            assert b[0] == 0 and b[-1] == n
            assert all(x < y for x, y in zip(b, b[1:]))
            assert len(b) - 1 == min(want, n)
            if len(b) == 3:
                assert b[1] >= n - b[1]
    gm.set_split_streams(0)
    gm.set_schedule(ms.SCHED_FUSED)
    assert gm.split_parts(4096) == [0, 4096]
