"""The geometry surrogate on the GPU, against the FP64 oracle.

* Network kernels (bfloat16 matrix-core GEMMs, SiLU, loss, backward, Adam)
  against the oracle network evaluated with the same bfloat16 rounding
  points.
* The surrogate step: an env whose predictions pass the checks advances as
  the oracle step given the predicted geometry; an env that fails them
  advances exactly as the exact path does (bit for bit) and is flagged.

Poses are drawn on the host from seeded generators; targets, moment-arm
spans and expected states come from the oracle.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_2603_29332_amd import ms, synth  # noqa: E402

DEV = "cuda"


def _t(a, dtype=torch.float32):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


@pytest.fixture(scope="module")
def setup():
    m = synth.chain_model(1)
    gm = ms.Model(m)
    s = ms.Surrogate(gm, hidden=64, seed=5)
    return m, gm, s, oracle.Oracle(m)


def _oracle_spans(m, o):
    """DoFs each muscle's length depends on (ascending, -1 padded to 3),
    read off the oracle's moment arms at two random poses."""
    rng = np.random.default_rng(77)
    nz = np.zeros((m["n_mus"], m["nv"]), bool)
    for _ in range(2):
        q = rng.uniform(-1, 1, m["nq"])
        _, r, _ = o.geometry(q, np.zeros(m["nv"]))
        nz |= np.abs(r) > 1e-12
    sp = -np.ones((m["n_mus"], 3), np.int64)
    for k in range(m["n_mus"]):
        j = np.flatnonzero(nz[k])
        assert j.size <= 3
        sp[k, :j.size] = j
    return sp


def _oracle_targets(m, o, spans, q):
    """[L | r in span slots] per pose from the oracle's geometry."""
    n = q.shape[0]
    y = np.zeros((n, 4 * m["n_mus"]))
    for p in range(n):
        L, r, _ = o.geometry(q[p], np.zeros(m["nv"]))
        y[p, :m["n_mus"]] = L
        for k in range(m["n_mus"]):
            for sl in range(3):
                if spans[k, sl] >= 0:
                    y[p, m["n_mus"] + 3 * k + sl] = r[k, spans[k, sl]]
    return y


def _full_r(m, spans, rs):
    """Moment arms in span slots -> [n_mus][nv]."""
    r = np.zeros((m["n_mus"], m["nv"]))
    for k in range(m["n_mus"]):
        for sl in range(3):
            if spans[k, sl] >= 0:
                r[k, spans[k, sl]] = rs[k, sl]
    return r


def _poses(m, n, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(m["qlo"], m["qhi"], (n, m["nq"])).astype(np.float32)


def _oracle_params(ps):
    """GPU stores W as [out][in]; the oracle takes [in][out]."""
    W1, b1, W2, b2, W3, b3 = ps
    return [W1.T.copy(), b1, W2.T.copy(), b2, W3.T.copy(), b3]


def _inputs(m, s, q):
    """Network inputs of poses q: each hinge angle mapped from its pose box
    onto [-1, 1] in float32 as the library defines it, zero-padded."""
    lo = np.asarray(m["qlo"], np.float32)
    hi = np.asarray(m["qhi"], np.float32)
    c = np.float32(0.5) * (lo + hi)
    isc = np.float32(2.0) / (hi - lo)
    x = np.zeros((q.shape[0], s.n_in), np.float32)
    x[:, :m["nq"]] = (np.asarray(q, np.float32) - c) * isc
    return x


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)


def _identity_norm(s):
    s.set_norm(np.zeros(s.n_out, np.float32), np.ones(s.n_out, np.float32))


def test_forward_matches_oracle(setup):
    m, gm, s, o = setup
    rng = np.random.default_rng(0)
    ps = s.params()
    ps[1][:] = rng.normal(size=ps[1].shape) * 0.1
    ps[3][:] = rng.normal(size=ps[3].shape) * 0.1
    ps[5][:] = rng.normal(size=ps[5].shape) * 0.1
    s.set_params(ps)
    mean = rng.normal(size=s.n_out).astype(np.float32)
    std = rng.uniform(0.5, 2, s.n_out).astype(np.float32)
    s.set_norm(mean, std)
    n = 136                                     # two 128-row tiles, ragged
    qh = _poses(m, n, 9)
    q = _t(qh)
    L = torch.zeros(n, m["n_mus"], device=DEV)
    r = torch.zeros(n, m["n_mus"], 3, device=DEV)
    s.forward(q, L, r)
    torch.cuda.synchronize()
    y = np.concatenate([L.cpu().numpy(), r.cpu().numpy().reshape(n, -1)], axis=1)
    yo = oracle.mlp_forward(_oracle_params(ps), _inputs(m, s, qh), bf16=True) * std + mean
    assert _rel(y, yo) < 2e-3
    _identity_norm(s)


def test_gradients_match_oracle(setup):
    m, gm, s, o = setup
    n = 64
    qh = _poses(m, n, 3)
    spans = _oracle_spans(m, o)
    t = _oracle_targets(m, o, spans, qh).astype(np.float32)
    L = _t(t[:, :m["n_mus"]])
    r = _t(t[:, m["n_mus"]:].reshape(n, m["n_mus"], 3))
    loss = torch.zeros(1, device=DEV)
    s.train_step(_t(qh), L, r, lr=0.0, step=1, loss=loss)
    torch.cuda.synchronize()
    g = s.grads()
    ps = s.params()
    mask = np.ones(s.n_out, np.float32)
    mask[m["n_mus"]:] = (spans.reshape(-1) >= 0)
    lo, go = oracle.mlp_grad(_oracle_params(ps), _inputs(m, s, qh), t * mask,
                             np.tile(mask, (n, 1)), bf16=True)
    assert abs(loss.item() - lo) < 1e-3 * lo
    pairs = [(g[0], go[0].T), (g[1], go[1]), (g[2], go[2].T), (g[3], go[3]), (g[4], go[4].T),
             (g[5], go[5])]
    for k, (a, b) in enumerate(pairs):
        assert _rel(a, b) < 1e-2, (k, _rel(a, b))


def test_adam_update_matches_oracle(setup):
    m, gm, s, o = setup
    n = 32
    qh = _poses(m, n, 4)
    spans = _oracle_spans(m, o)
    t = _oracle_targets(m, o, spans, qh).astype(np.float32)
    L = _t(t[:, :m["n_mus"]])
    r = _t(t[:, m["n_mus"]:].reshape(n, m["n_mus"], 3))
    p0 = s.params()
    s.train_step(_t(qh), L, r, lr=1e-3, step=1)
    torch.cuda.synchronize()
    g = s.grads()
    p1 = s.params()
    for a, b, gg in zip(p0, p1, g):
        w = a.astype(np.float64).copy()
        mm = np.zeros_like(w)
        vv = np.zeros_like(w)
        oracle.adam(w.reshape(-1), mm.reshape(-1), vv.reshape(-1), gg.astype(np.float64).reshape(-1),
                    lr=1e-3, step=1)
        assert np.abs(b - w).max() < 1e-6


def test_sampled_poses_lie_in_the_box(setup):
    m, gm, s, o = setup
    q = torch.zeros(1000, m["nq"], device=DEV)
    s.sample(q, seed=1, offset=5)
    q2 = torch.zeros(1000, m["nq"], device=DEV)
    s.sample(q2, seed=1, offset=5)
    torch.cuda.synchronize()
    qa = q.cpu().numpy()
    assert np.array_equal(qa, q2.cpu().numpy())
    assert (qa >= m["qlo"]).all() and (qa <= m["qhi"]).all()
    assert qa.std(axis=0).min() > 1.0        # spread over +-pi


# ------------------------------------------------------------ surrogate step
def _constant_network(m, s, o, spans, q_ref, r_scale=None):
    """Zero the output layer so the network returns exactly its shift: the
    oracle geometry at q_ref with lengths and the moment arms of the span
    slots 0.5 mm long (wrong enough to tell apart from the exact geometry,
    close enough to pass a 1 mm check of lengths and moment arms), or with
    exact lengths and the moment arms scaled by r_scale. Returns (L, r
    slots) as float32."""
    ps = s.params()
    ps[4][:] = 0.0
    ps[5][:] = 0.0
    s.set_params(ps)
    y = _oracle_targets(m, o, spans, q_ref[None])[0]
    if r_scale is None:
        y[:m["n_mus"]] += 5e-4
        y[m["n_mus"]:] += 5e-4 * (spans.reshape(-1) >= 0)
    else:
        y[m["n_mus"]:] *= r_scale
    y = y.astype(np.float32)
    s.set_norm(y, np.ones(s.n_out, np.float32))
    return y[:m["n_mus"]], y[m["n_mus"]:].reshape(m["n_mus"], 3)


def _states(m, E, q_ref, near, seed):
    rng = np.random.default_rng(seed)
    q = np.tile(q_ref, (E, 1)).astype(np.float32)
    far = ~near
    q[near] += rng.uniform(-2e-6, 2e-6, (near.sum(), m["nq"])).astype(np.float32)
    q[far] += rng.uniform(0.2, 0.4, (far.sum(), m["nq"])).astype(np.float32)
    qd = rng.normal(0, 0.3, (E, m["nv"])).astype(np.float32)
    act = rng.uniform(0.05, 0.6, (E, m["n_mus"])).astype(np.float32)
    return q, qd, act


def test_surrogate_step_matches_oracle_given_geometry_and_falls_back(setup):
    m, gm, s, o = setup
    spans = _oracle_spans(m, o)
    q_ref = np.linspace(-0.4, 0.4, m["nq"])
    Lr, rr = _constant_network(m, s, o, spans, q_ref)
    E, dt = 96, 2e-3
    near = np.arange(E) % 3 != 0
    q, qd, act = _states(m, E, q_ref, near, 5)
    u = synth.excitation_iid(12, E, m["n_mus"], 0)
    tq, tqd, tact = _t(q), _t(qd), _t(act)
    st = torch.zeros(E, dtype=torch.int32, device=DEV)
    fb = torch.zeros(E, dtype=torch.int32, device=DEV)
    gm.rollout_surrogate(s, tq, tqd, tact, st, 1, dt, contact=False, tol=1e-3,
                         fb_count=fb, kind=ms.EXC_ARRAY, u=_t(u[None]))
    # the exact path on the same states
    eq, eqd, eact = _t(q), _t(qd), _t(act)
    est = torch.zeros(E, dtype=torch.int32, device=DEV)
    gm.rollout(eq, eqd, eact, est, 1, dt, False, kind=ms.EXC_ARRAY, u=_t(u[None]))
    torch.cuda.synchronize()
    st, fb = st.cpu().numpy(), fb.cpu().numpy()
    assert (est.cpu().numpy() == 0).all()
    assert np.array_equal(fb, (~near).astype(np.int32))
    assert np.array_equal(st, np.where(near, 0, ms.MS_ST_FALLBACK))
    g = [x.cpu().numpy() for x in (tq, tqd, tact)]
    ex = [x.cpu().numpy() for x in (eq, eqd, eact)]
    for a, b in zip(g, ex):
        assert np.array_equal(a[~near], b[~near])
    rfull = _full_r(m, spans, rr)
    for e in np.flatnonzero(near):
        qo, qdo, ao, sto = o.step(dt, q[e], qd[e], act[e], u[e], contact=False,
                                  geometry=(Lr, rfull))
        assert sto == 0
        for a, b in zip((g[0][e], g[1][e], g[2][e]), (qo, qdo, ao)):
            assert np.abs(a - b).max() / max(np.abs(b).max(), 1.0) <= 1e-5
    # the predicted geometry is not the exact one: near envs differ from the
    # exact path
    assert np.abs(g[1][near] - ex[1][near]).max() > 1e-3
    _identity_norm(s)


def test_moment_arm_sentinel_sends_envs_to_the_exact_path(setup):
    """Exact lengths but moment arms 50 % large: every sentinel length passes
    a 1 mm check, so only the moment-arm check can send the envs near the
    reference pose to the exact geometry; they then advance bit for bit as
    the exact path does."""
    m, gm, s, o = setup
    spans = _oracle_spans(m, o)
    q_ref = np.linspace(-0.4, 0.4, m["nq"])
    _constant_network(m, s, o, spans, q_ref, r_scale=1.5)
    E, dt = 48, 2e-3
    near = np.ones(E, bool)
    q, qd, act = _states(m, E, q_ref, near, 7)
    u = synth.excitation_iid(14, E, m["n_mus"], 0)
    tq, tqd, tact = _t(q), _t(qd), _t(act)
    st = torch.zeros(E, dtype=torch.int32, device=DEV)
    fb = torch.zeros(E, dtype=torch.int32, device=DEV)
    gm.rollout_surrogate(s, tq, tqd, tact, st, 1, dt, contact=False, tol=1e-3,
                         fb_count=fb, kind=ms.EXC_ARRAY, u=_t(u[None]))
    eq, eqd, eact = _t(q), _t(qd), _t(act)
    est = torch.zeros(E, dtype=torch.int32, device=DEV)
    gm.rollout(eq, eqd, eact, est, 1, dt, False, kind=ms.EXC_ARRAY, u=_t(u[None]))
    torch.cuda.synchronize()
    assert (fb.cpu().numpy() == 1).all()
    assert (st.cpu().numpy() == ms.MS_ST_FALLBACK).all()
    for a, b in zip((tq, tqd, tact), (eq, eqd, eact)):
        assert torch.equal(a, b)
    _identity_norm(s)


def test_surrogate_rollout_with_negative_tolerance_is_the_exact_path(setup):
    m, gm, s, o = setup
    E, T, dt = 64, 5, 2e-3
    q, qd, act = synth.chain_initial_state(m, E, seed=3)
    x0 = np.zeros((E, m["n_mus"]), np.float32)
    runs = []
    for sur in (True, False):
        tq, tqd, tact, tx = _t(q), _t(qd), _t(act), _t(x0)
        st = torch.zeros(E, dtype=torch.int32, device=DEV)
        fb = torch.zeros(E, dtype=torch.int32, device=DEV)
        consts = synth.ar1_constants(dt)[:3]
        if sur:
            gm.rollout_surrogate(s, tq, tqd, tact, st, T, dt, contact=False, tol=-1.0,
                                 fb_count=fb, kind=ms.EXC_AR1, seed=4, step0=2, x=tx,
                                 ar1=consts)
        else:
            gm.rollout(tq, tqd, tact, st, T, dt, False, kind=ms.EXC_AR1, seed=4, step0=2, x=tx,
                       ar1=consts)
        torch.cuda.synchronize()
        runs.append([v.cpu().numpy() for v in (tq, tqd, tact, tx, st, fb)])
    a, b = runs
    for k in range(4):
        assert np.array_equal(a[k], b[k])
    assert (a[4] == ms.MS_ST_FALLBACK).all() and (b[4] == 0).all()
    assert (a[5] == T).all()


def test_training_gain_fewer_fallbacks_and_smaller_error():
    """What training gains, on the chain model: the network trained by the
    library's own kernels (1500 Adam iterations of 8192 sampled poses)
    predicts the oracle's muscle lengths on held-out poses far better than
    the same network untrained, and in a rollout whose residual check allows
    1 cm it replaces the exact geometry on almost every step, where the
    untrained network falls back on every step."""
    from paper_2603_29332_amd import surrogate
    m = synth.chain_model(1)
    gm = ms.Model(m)
    o = oracle.Oracle(m)
    q = _poses(m, 96, 2025)
    Lo = np.array([o.geometry(q[p].astype(np.float64), np.zeros(m["nv"]))[0]
                   for p in range(len(q))])
    dt = 2e-3
    rho, sd, mean_u, _ = synth.ar1_constants(dt)

    def error_and_fallback(sg):
        L = torch.empty(len(q), m["n_mus"], device=DEV)
        r = torch.empty(len(q), m["n_mus"], 3, device=DEV)
        sg.forward(_t(q), L, r)
        torch.cuda.synchronize()
        err = float(np.median(np.abs(L.cpu().numpy() - Lo).max(axis=1)))
        E = 512
        q0, qd0, a0 = synth.chain_initial_state(m, E)
        tq, tqd, ta = _t(q0), _t(qd0), _t(a0)
        st = torch.zeros(E, dtype=torch.int32, device=DEV)
        fb = torch.zeros(E, dtype=torch.int32, device=DEV)
        x = torch.zeros(E, m["n_mus"], device=DEV)
        gm.rollout_surrogate(sg, tq, tqd, ta, st, 100, dt, False, tol=1e-2, fb_count=fb,
                             kind=ms.EXC_AR1, seed=5, x=x, ar1=(rho, sd, mean_u))
        torch.cuda.synchronize()
        return err, fb.sum().item() / (E * 100)

    untrained = ms.Surrogate(gm, hidden=512, seed=41)
    untrained.train(iters=0, norm_samples=8192)       # output standardisation only
    e0, f0 = error_and_fallback(untrained)
    trained = ms.Surrogate(gm, hidden=512, seed=41)
    surrogate.train(trained, n_samples=10_000_000, batch=8192, epochs=1500 * 8192 / 10_000_000)
    e1, f1 = error_and_fallback(trained)
    print(f"median worst-muscle length error {e0:.4f} m untrained, {e1:.4f} m trained; "
          f"fallback rate at 1 cm {f0:.3f} untrained, {f1:.3f} trained")
    assert e1 <= 0.1 * e0 and e1 <= 1e-2
    assert f0 >= 0.95 and f1 <= 0.05


def test_save_and_load_reproduce_the_network(setup, tmp_path):
    """A network written by save() and read into a fresh one with load()
    predicts bit for bit the same lengths and moment arms."""
    m, gm, s, o = setup
    rng = np.random.default_rng(31)
    s.set_params([rng.normal(0, 0.3, sh).astype(np.float32) for sh in s.shapes])
    s.set_norm(rng.normal(0, 0.1, s.n_out).astype(np.float32),
               rng.uniform(0.5, 2.0, s.n_out).astype(np.float32))
    path = tmp_path / "net.msg"
    s.save(path)
    s2 = ms.Surrogate(gm, hidden=s.h1, seed=99)
    s2.load(path)
    q = _t(_poses(m, 40, 12))
    outs = []
    for net in (s, s2):
        L = torch.empty(40, m["n_mus"], device=DEV)
        r = torch.empty(40, m["n_mus"], 3, device=DEV)
        net.forward(q, L, r)
        outs.append((L, r))
    torch.cuda.synchronize()
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
    for a, b in zip(s.params(), s2.params()):
        assert np.array_equal(a, b)


def test_full_size_surrogate_rollout_falls_back_to_the_exact_path():
    """The surrogate workload at its full size (whole body, 4096 envs, AR(1)
    excitations in-kernel, 1e-4 m residual check): a network that fails the
    check everywhere (untrained) sends every env-step to the exact geometry,
    and the rollout is the exact path's, bit for bit."""
    m = synth.human_model(2)
    gm = ms.Model(m)
    s = ms.Surrogate(gm, hidden=512, seed=41)
    E, T, dt = 4096, 10, 1e-3
    q, qd, act = synth.human_initial_state(m, E)
    consts = synth.ar1_constants(dt)[:3]
    runs = []
    for sur in (True, False):
        tq, tqd, tact = _t(q), _t(qd), _t(act)
        tx = torch.zeros(E, m["n_mus"], device=DEV)
        st = torch.zeros(E, dtype=torch.int32, device=DEV)
        fb = torch.zeros(E, dtype=torch.int32, device=DEV)
        if sur:
            gm.rollout_surrogate(s, tq, tqd, tact, st, T, dt, True, tol=1e-4, fb_count=fb,
                                 kind=ms.EXC_AR1, seed=12, x=tx, ar1=consts)
        else:
            gm.rollout(tq, tqd, tact, st, T, dt, True, kind=ms.EXC_AR1, seed=12, x=tx, ar1=consts)
        torch.cuda.synchronize()
        runs.append([v.cpu().numpy() for v in (tq, tqd, tact, tx, st, fb)])
    a, b = runs
    for k in range(4):
        assert np.array_equal(a[k], b[k])
    assert ((a[4] & ~ms.MS_ST_FALLBACK) == b[4]).all()
    assert (a[5] == T).all()


# ------------------------------------------------- whole-body network, full size
def _hinge_inputs(m):
    """q index and pose box of every network input (hinge/slide coordinates
    in node order; a free root's seven coordinates are not inputs)."""
    qi, lo, hi = [], [], []
    qa = da = 0
    for i in range(m["n_node"]):
        if m["jtype"][i] == 2:
            qa, da = qa + 7, da + 6
            continue
        qi.append(qa)
        lo.append(m["qlo"][da])
        hi.append(m["qhi"][da])
        qa, da = qa + 1, da + 1
    return np.array(qi), np.asarray(lo, np.float32), np.asarray(hi, np.float32)


def _human_poses(m, n, seed):
    """Hinge coordinates uniform in their boxes; the root at the origin with
    the identity orientation."""
    qi, lo, hi = _hinge_inputs(m)
    rng = np.random.default_rng(seed)
    q = np.zeros((n, m["nq"]), np.float32)
    q[:, 3] = 1.0
    q[:, qi] = rng.uniform(lo, hi, (n, len(qi))).astype(np.float32)
    return q


def _human_inputs(m, s, q):
    qi, lo, hi = _hinge_inputs(m)
    c = np.float32(0.5) * (lo + hi)
    isc = np.float32(2.0) / (hi - lo)
    x = np.zeros((q.shape[0], s.n_in), np.float32)
    x[:, :len(qi)] = (q[:, qi] - c) * isc
    return x


@pytest.fixture(scope="module")
def human_net():
    m = synth.human_model(2)
    gm = ms.Model(m)
    o = oracle.Oracle(m)
    s = ms.Surrogate(gm, hidden=512, seed=41)
    spans = _oracle_spans(m, o)
    assert np.array_equal(gm.spans(), spans)
    return m, gm, s, o, spans


@pytest.mark.parametrize("n", [2048, 2056])
def test_full_size_network_forward_gradients_and_adam(human_net, n):
    """The whole-body network (74 inputs padded to 80 -> 512 -> 512 -> 2800)
    at batch 2048, so every GEMM runs several M, N and K tiles and the
    weight gradients run split-K with several slices, and at 2056, whose
    last row tile, last 64-row loss chunk and last K slice are ragged:
    forward outputs, the loss, all six gradients, one Adam step, and the
    gradients again with the updated weights (the transposed weight copies
    the backward products read are refreshed by the Adam step), against the
    oracle network with the same bfloat16 rounding points."""
    m, gm, _, o, spans = human_net
    s = ms.Surrogate(gm, hidden=512, seed=41)   # fresh Adam moments for the step below
    rng = np.random.default_rng(n)
    ps = s.params()
    for k in (1, 3, 5):
        ps[k][:] = rng.normal(size=ps[k].shape) * 0.1
    s.set_params(ps)
    qh = _human_poses(m, n, 17)
    x = _human_inputs(m, s, qh)
    # forward, de-standardised
    mean = rng.normal(size=s.n_out).astype(np.float32)
    std = rng.uniform(0.5, 2, s.n_out).astype(np.float32)
    s.set_norm(mean, std)
    L = torch.zeros(n, m["n_mus"], device=DEV)
    r = torch.zeros(n, m["n_mus"], 3, device=DEV)
    s.forward(_t(qh), L, r)
    torch.cuda.synchronize()
    y = np.concatenate([L.cpu().numpy(), r.cpu().numpy().reshape(n, -1)], axis=1)
    yo = oracle.mlp_forward(_oracle_params(ps), x, bf16=True) * std + mean
    assert _rel(y, yo) < 2e-3, _rel(y, yo)
    # gradients on random targets (identity standardisation)
    _identity_norm(s)
    t = rng.normal(0, 0.5, (n, s.n_out)).astype(np.float32)
    mask = np.ones(s.n_out, np.float32)
    mask[m["n_mus"]:] = (spans.reshape(-1) >= 0)
    t *= mask
    loss = torch.zeros(1, device=DEV)
    s.train_step(_t(qh), _t(t[:, :m["n_mus"]]), _t(t[:, m["n_mus"]:].reshape(n, m["n_mus"], 3)),
                 lr=0.0, step=1, loss=loss)
    torch.cuda.synchronize()
    g = s.grads()
    lo, go = oracle.mlp_grad(_oracle_params(ps), x, t, np.tile(mask, (n, 1)), bf16=True)
    assert abs(loss.item() - lo) < 1e-3 * lo, (loss.item(), lo)
    pairs = [(g[0], go[0].T), (g[1], go[1]), (g[2], go[2].T), (g[3], go[3]), (g[4], go[4].T),
             (g[5], go[5])]
    for k, (a, b) in enumerate(pairs):
        assert _rel(a, b) < 1e-2, (k, _rel(a, b))
    # one Adam step on the same batch
    p0 = s.params()
    s.train_step(_t(qh), _t(t[:, :m["n_mus"]]), _t(t[:, m["n_mus"]:].reshape(n, m["n_mus"], 3)),
                 lr=1e-3, step=1)
    torch.cuda.synchronize()
    g1 = s.grads()
    p1 = s.params()
    for a, b, gg in zip(p0, p1, g1):
        w = a.astype(np.float64).copy()
        mm = np.zeros_like(w)
        vv = np.zeros_like(w)
        oracle.adam(w.reshape(-1), mm.reshape(-1), vv.reshape(-1),
                    gg.astype(np.float64).reshape(-1), lr=1e-3, step=1)
        assert np.abs(b - w).max() < 1e-6
    # gradients at the updated weights
    s.train_step(_t(qh), _t(t[:, :m["n_mus"]]), _t(t[:, m["n_mus"]:].reshape(n, m["n_mus"], 3)),
                 lr=0.0, step=2)
    torch.cuda.synchronize()
    g2 = s.grads()
    _, go2 = oracle.mlp_grad(_oracle_params(p1), x, t, np.tile(mask, (n, 1)), bf16=True)
    pairs = [(g2[0], go2[0].T), (g2[1], go2[1]), (g2[2], go2[2].T), (g2[3], go2[3]),
             (g2[4], go2[4].T), (g2[5], go2[5])]
    for k, (a, b) in enumerate(pairs):
        assert _rel(a, b) < 1e-2, (k, _rel(a, b))


def test_full_size_prediction_taken_step_matches_oracle(human_net):
    """Whole body, contact off: a constant network returning the oracle's
    geometry at a reference pose (lengths and moment arms 0.5 mm long)
    passes a 1 mm residual check on envs within 2e-6 of that pose,
    which then advance as the oracle step given that geometry (per-step
    bound 1e-5); envs moved 0.2-0.4 rad away fail it and advance bit for bit
    as the exact path does."""
    m, gm, s, o, spans = human_net
    qi, _, _ = _hinge_inputs(m)
    q0, _, _ = synth.human_initial_state(m, 1, seed=21)
    q_ref = q0[0].astype(np.float64)
    Lr, rr = _constant_network(m, s, o, spans, q_ref)
    E, dt = 128, 1e-3
    near = np.arange(E) % 4 != 0
    rng = np.random.default_rng(6)
    q = np.tile(q_ref, (E, 1)).astype(np.float32)
    q[np.ix_(near, qi)] += rng.uniform(-2e-6, 2e-6, (near.sum(), len(qi))).astype(np.float32)
    q[np.ix_(~near, qi)] += rng.uniform(0.2, 0.4, ((~near).sum(), len(qi))).astype(np.float32)
    qd = rng.normal(0, 0.3, (E, m["nv"])).astype(np.float32)
    act = rng.uniform(0.05, 0.6, (E, m["n_mus"])).astype(np.float32)
    u = synth.excitation_iid(13, E, m["n_mus"], 0)
    tq, tqd, tact = _t(q), _t(qd), _t(act)
    st = torch.zeros(E, dtype=torch.int32, device=DEV)
    fb = torch.zeros(E, dtype=torch.int32, device=DEV)
    gm.rollout_surrogate(s, tq, tqd, tact, st, 1, dt, contact=False, tol=1e-3,
                         fb_count=fb, kind=ms.EXC_ARRAY, u=_t(u[None]))
    eq, eqd, eact = _t(q), _t(qd), _t(act)
    est = torch.zeros(E, dtype=torch.int32, device=DEV)
    gm.rollout(eq, eqd, eact, est, 1, dt, False, kind=ms.EXC_ARRAY, u=_t(u[None]))
    torch.cuda.synchronize()
    st, fb = st.cpu().numpy(), fb.cpu().numpy()
    assert (est.cpu().numpy() == 0).all()
    assert np.array_equal(fb, (~near).astype(np.int32))
    assert np.array_equal(st, np.where(near, 0, ms.MS_ST_FALLBACK))
    g = [x.cpu().numpy() for x in (tq, tqd, tact)]
    ex = [x.cpu().numpy() for x in (eq, eqd, eact)]
    for a, b in zip(g, ex):
        assert np.array_equal(a[~near], b[~near])
    rfull = _full_r(m, spans, rr)
    worst = 0.0
    for e in np.flatnonzero(near)[::6]:
        qo, qdo, ao, sto = o.step(dt, q[e], qd[e], act[e], u[e], contact=False,
                                  geometry=(Lr, rfull))
        assert sto == 0
        for a, b in zip((g[0][e], g[1][e], g[2][e]), (qo, qdo, ao)):
            err = np.abs(a - b).max() / max(np.abs(b).max(), 1.0)
            worst = max(worst, err)
            assert err <= 1e-5, (e, err)
    print(f"prediction-taken whole-body step: worst per-block error {worst:.2e}")
    assert np.abs(g[1][near] - ex[1][near]).max() > 1e-3
    _identity_norm(s)


# ------------------------------------------------ training behind the C ABI
def _host_poses(m, seed, offset, n, n_in):
    """Poses of the library's pose sampler regenerated on the host from its
    published definition: input i of pose p is lo + (hi - lo) u with u the
    top 24 bits x 2^-24 of SplitMix64(SplitMix64(seed ^ (offset + p)) ^ i)."""
    M = (1 << 64) - 1

    def sm(x):
        z = (x + 0x9E3779B97F4A7C15) & M
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        return z ^ (z >> 31)

    qi, lo, hi = _hinge_inputs(m) if m["jtype"][0] == 2 else (
        np.arange(m["nq"]), np.asarray(m["qlo"], np.float32), np.asarray(m["qhi"], np.float32))
    q = np.zeros((n, m["nq"]), np.float32)
    if m["jtype"][0] == 2:
        q[:, 3] = 1.0
    for p in range(n):
        key = sm(seed ^ (offset + p))
        for i in range(len(qi)):
            u = np.float32((sm(key ^ i) >> 40) * 5.9604644775390625e-8)
            q[p, qi[i]] = np.float32(lo[i] + np.float32(hi[i] - lo[i]) * u)
    return q


def _blob(path, s):
    """Layer sizes, weights and standardisation from a saved blob."""
    raw = open(path, "rb").read()
    head = np.frombuffer(raw[:32], np.uint32)
    assert head[0] == 0x4D534731 and head[1] == 1
    n_in, h1, h2, n_out = (int(x) for x in head[2:6])
    body = np.frombuffer(raw[32:], np.float32)
    sizes = [h1 * n_in, h1, h2 * h1, h2, n_out * h2, n_out, n_out, n_out]
    assert body.size == sum(sizes)
    parts, o = [], 0
    for k in sizes:
        parts.append(body[o:o + k])
        o += k
    return (n_in, h1, h2, n_out), parts


def test_train_sets_the_standardisation_of_oracle_labels(tmp_path):
    """ms_surrogate_train with no steps sets each output's mean and standard
    deviation over the sampled poses; the oracle labels of the same poses
    (regenerated on the host) give the same statistics."""
    m = synth.chain_model(1)
    gm = ms.Model(m)
    o = oracle.Oracle(m)
    s = ms.Surrogate(gm, hidden=64, seed=7)
    n = 200
    s.train(iters=0, norm_samples=n, norm_seed=40, batch=64)
    s.save(tmp_path / "n.msg")
    dims, parts = _blob(tmp_path / "n.msg", s)
    mean, std = parts[6], parts[7]
    spans = _oracle_spans(m, o)
    q = _host_poses(m, 40, 0, n, s.n_in)
    y = _oracle_targets(m, o, spans, q.astype(np.float64))
    have = np.r_[np.ones(m["n_mus"], bool), spans.reshape(-1) >= 0]
    mo = y.mean(0)
    so = np.sqrt(((y - mo) ** 2).mean(0))
    assert np.abs(mean[have] - mo[have]).max() < 2e-6
    assert (np.abs(std[have] - so[have]) <= 1e-4 * so[have] + 2e-6).all()
    assert (mean[~have] == 0).all() and (std[~have] == 1).all()


def test_train_equals_its_steps_taken_one_by_one():
    """Three steps of ms_surrogate_train equal three ms_surrogate_train_step
    calls on the library's sampled poses and exact labels with the cosine
    learning rates, bit for bit, and the loss falls."""
    m = synth.chain_model(1)
    gm = ms.Model(m)
    B, iters, lr0, lr1 = 256, 3, 1e-2, 1e-5
    a = ms.Surrogate(gm, hidden=64, seed=8)
    b = ms.Surrogate(gm, hidden=64, seed=8)
    loss = torch.zeros(iters, device=DEV)
    a.train(n_samples=1000, batch=B, iters=iters, lr0=lr0, lr1=lr1, seed=41, norm_samples=512,
            loss=loss)
    b.train(iters=0, norm_samples=512, batch=B)
    q = torch.zeros(B, m["nq"], device=DEV)
    L = torch.zeros(B, m["n_mus"], device=DEV)
    r = torch.zeros(B, m["n_mus"], 3, device=DEV)
    for it in range(iters):
        b.sample(q, 41, (it * B) % 1000)
        gm.geometry(q, L, r)
        lr = np.float32(lr1 + 0.5 * (lr0 - lr1) * (1.0 + np.cos(np.pi * it / iters)))
        b.train_step(q, L, r, float(lr), it + 1)
    torch.cuda.synchronize()
    for x, y in zip(a.params(), b.params()):
        assert np.array_equal(x, y)
    lv = loss.cpu().numpy()
    assert np.isfinite(lv).all() and lv[-1] < lv[0]


def test_train_step_argument_bounds(setup):
    """Batches that are not a positive multiple of 8 or exceed 2^20 (the
    weight gradients take the batch as a row length), and step 0, are
    refused with MS_E_ARG before anything is read or launched."""
    m, gm, s, o = setup
    q = torch.zeros(8, m["nq"], device=DEV)
    L = torch.zeros(8, m["n_mus"], device=DEV)
    r = torch.zeros(8, m["n_mus"], 3, device=DEV)
    for n, step in ((0, 1), (12, 1), ((1 << 20) + 8, 1), (8, 0)):
        rc = ms.lib().ms_surrogate_train_step(s.h, n, ms._dp(q), ms._dp(L), ms._dp(r), 0.0, step,
                                              None, None)
        assert rc == -1, (n, step, rc)
    s.train_step(q, L, r, 0.0, 1)   # the smallest valid batch still runs
    torch.cuda.synchronize()
