"""Compliant tendons (ms_rollout_tendon) against the FP64 oracle's
compliant-tendon step, through the C ABI.

Tolerances:
* per step, teacher-forced, per state block x in {q, qd, act}:
  max|x_gpu - x_ora| / max(max|x_ora|, 1), and for the fibre lengths
  max|lm_gpu - lm_ora| / max|lm_ora|: within 1e-5, or within 4 times the
  oracle's own spread when every fibre length moves by 4 ulps (float32) of
  its path length, capped at 5e-4. The tendon turns the float32 rounding
  of the path length into a force error F0 dL / (eps0 l_slack), 1 / eps0 =
  30 times the rigid fibre's sensitivity to the same rounding, and the
  velocities follow it: the first run against a literal 1e-5 on the chain
  found velocity errors of 2e-6 to 1.13e-5 (3 of 16 states above 1e-5)
  with lengths, positions and activations within 4e-7. The number of
  states above 1e-5 is printed;
* free run: max |q_gpu - q_ora| <= 1e-3 rad after 200 steps (chain).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import Oracle  # noqa: E402
from paper_2603_29332_amd import ms, synth  # noqa: E402
from tests import models  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda"
EPS0, BETA = 0.033, 0.1
CAP = 5e-4


def _t(a, dtype=torch.float32):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


@pytest.fixture(scope="module")
def chain():
    m = synth.chain_model(1)
    return m, ms.Model(m), Oracle(m)


@pytest.fixture(scope="module")
def human():
    m = synth.human_model(2)
    return m, ms.Model(m), Oracle(m)


def _initial(m, o, init, E):
    """Seeded states; fibres at the length that leaves each tendon 0.5 %
    above slack (path lengths from the oracle's geometry)."""
    q, qd, act = (np.asarray(v, np.float64) for v in init(m, E))
    L = np.stack([o.geometry(q[e], qd[e])[0] for e in range(E)])
    lm = L - np.asarray(m["l_slack"], np.float64) * 1.005
    return q, qd, act, lm


def _oracle_steps(o, dt, q, qd, act, lm, us, contact):
    q, qd, act, lm = q.copy(), qd.copy(), act.copy(), lm.copy()
    for u in us:
        for e in range(q.shape[0]):
            q[e], qd[e], act[e], lm[e], st = o.step_tendon(dt, q[e], qd[e], act[e], lm[e], u[e],
                                                          EPS0, BETA, contact=contact)
            assert st == 0
    return q, qd, act, lm


def _gpu_steps(gm, q, qd, act, lm, us, dt, contact, status=None):
    E = q.shape[0]
    a = [_t(q), _t(qd), _t(act), _t(lm)]
    st = torch.zeros(E, dtype=torch.int32, device=DEV) if status is None else _t(status, torch.int32)
    gm.rollout_tendon(*a, st, len(us), dt, contact, eps0=EPS0, beta=BETA, kind=ms.EXC_ARRAY,
                      u=_t(np.asarray(us, np.float32)))
    torch.cuda.synchronize()
    return [v.cpu().numpy() for v in a] + [st.cpu().numpy()]


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1.0)


def _warm(m, o, init, E, n, dt, contact):
    q, qd, act, lm = _initial(m, o, init, E)
    us = [synth.excitation_iid(22, E, m["n_mus"], t) for t in range(n)]
    q, qd, act, lm = _oracle_steps(o, dt, q, qd, act, lm, us, contact)
    return [v.astype(np.float32) for v in (q, qd, act, lm)]


@pytest.mark.parametrize("which", ["chain", "human"])
def test_tendon_step_teacher_forced(which, chain, human):
    """One GPU step from warmed-up float32 states (tendons taut, fibres
    moving) against the oracle's step."""
    m, gm, o = chain if which == "chain" else human
    init = synth.chain_initial_state if which == "chain" else synth.human_initial_state
    dt, E = (2e-3, 16) if which == "chain" else (1e-3, 12)
    q, qd, act, lm = _warm(m, o, init, E, 30, dt, False)
    u = synth.excitation_iid(6, E, m["n_mus"], 0)
    g = _gpu_steps(gm, q, qd, act, lm, [u], dt, False)
    assert (g[4] == 0).all()
    ref = _oracle_steps(o, dt, *(v.astype(np.float64) for v in (q, qd, act, lm)), [u], False)
    err = np.array([[_rel(g[0][e], ref[0][e]), _rel(g[1][e], ref[1][e]), _rel(g[2][e], ref[2][e]),
                     np.abs(g[3][e] - ref[3][e]).max() / np.abs(ref[3][e]).max()]
                    for e in range(E)])
    # the oracle's own spread when each fibre length moves by 4 ulps
    # (float32) of its path length
    spread = np.zeros(err.shape)
    L = np.stack([o.geometry(q[e].astype(np.float64), qd[e].astype(np.float64))[0]
                  for e in range(E)])
    ulp = np.spacing(L.astype(np.float32)).astype(np.float64)
    rng = np.random.default_rng(5)
    for _ in range(3):
        lp = lm.astype(np.float64) + 4 * ulp * rng.choice([-1.0, 1.0], size=lm.shape)
        p = _oracle_steps(o, dt, *(v.astype(np.float64) for v in (q, qd, act)), lp, [u], False)
        spread = np.maximum(spread, np.array(
            [[_rel(p[0][e], ref[0][e]), _rel(p[1][e], ref[1][e]), _rel(p[2][e], ref[2][e]),
              np.abs(p[3][e] - ref[3][e]).max() / np.abs(ref[3][e]).max()]
             for e in range(E)]))
    tol = np.clip(4 * spread, 1e-5, CAP)
    print(f"{which} tendon teacher-forced: max rel err (q, qd, act, lm) {err.max(axis=0)}; "
          f"{int((err > 1e-5).any(axis=1).sum())} of {E} states above 1e-5; oracle spread up to "
          f"{spread.max(axis=0)}; largest error / bound {(err / tol).max():.2f}")
    assert (err <= tol).all()


def test_tendon_freerun_chain_200(chain):
    """200 steps from the initial states, GPU against the oracle, every env
    within 1e-3 rad on every hinge."""
    m, gm, o = chain
    E, dt = 32, 2e-3
    q, qd, act, lm = _initial(m, o, synth.chain_initial_state, E)
    q, qd, act, lm = (v.astype(np.float32) for v in (q, qd, act, lm))
    us = [synth.excitation_iid(31, E, m["n_mus"], t) for t in range(200)]
    g = _gpu_steps(gm, q, qd, act, lm, us, dt, False)
    assert (g[4] == 0).all()
    ref = _oracle_steps(o, dt, *(v.astype(np.float64) for v in (q, qd, act, lm)), us, False)
    err = np.abs(g[0] - ref[0]).max()
    lerr = np.abs(g[3] - ref[3]).max()
    moved = np.abs(ref[0] - q).max()
    print(f"chain tendon 200 steps: max |dq| {err:.2e} rad, max |dlm| {lerr:.2e} m, "
          f"max excursion {moved:.2f} rad")
    assert moved > 0.05
    assert err <= 1e-3


def test_tendon_stream_parts_equal_one_stream(human):
    """The whole body on two concurrent stream parts equals one stream,
    bitwise, and the slack tendons of a batch at rest stay inside the
    workload (every env applied, lengths finite)."""
    m, gm, o = human
    E, dt = 640, 1e-3
    q, qd, act = synth.human_initial_state(m, E)
    L = torch.empty(E, m["n_mus"], device=DEV)
    r = torch.empty(E, m["n_mus"], 3, device=DEV)
    gm.geometry(_t(q), L, r)
    lm0 = L - _t(m["l_slack"]) * 1.005
    out = []
    for parts in (1, 2):
        gm.set_split_streams(parts)
        a = [_t(q), _t(qd), _t(act), lm0.clone()]
        st = torch.zeros(E, dtype=torch.int32, device=DEV)
        x = torch.zeros(E, m["n_mus"], device=DEV)
        gm.rollout_tendon(*a, st, 20, dt, True, eps0=EPS0, beta=BETA, kind=ms.EXC_AR1, seed=12,
                          x=x, ar1=synth.ar1_constants(dt)[:3])
        torch.cuda.synchronize()
        out.append([v.cpu().numpy() for v in a] + [st.cpu().numpy()])
    gm.set_split_streams(0)
    for x1, x2 in zip(out[0], out[1]):
        assert np.array_equal(x1, x2)
    assert (out[0][4] == 0).all() and np.isfinite(out[0][3]).all()
    ln = out[0][3] / m["l_opt"]
    print(f"whole body, 20 steps with contact: fibre lengths {ln.min():.3f} .. {ln.max():.3f} l_opt")
    assert ln.min() > 0.3 and ln.max() < 2.0


def test_tendon_freerun_human_200_contact_off(human):
    """The whole body, 200 steps from its initial states with contact off,
    GPU against the oracle: every hinge within 1e-3 rad, the root within
    1e-3 m, the fibres within 1e-5 m."""
    m, gm, o = human
    E, dt = 6, 1e-3
    q, qd, act, lm = _initial(m, o, synth.human_initial_state, E)
    q, qd, act, lm = (v.astype(np.float32) for v in (q, qd, act, lm))
    us = [synth.excitation_iid(41, E, m["n_mus"], t) for t in range(200)]
    g = _gpu_steps(gm, q, qd, act, lm, us, dt, False)
    assert (g[4] == 0).all()
    ref = _oracle_steps(o, dt, *(v.astype(np.float64) for v in (q, qd, act, lm)), us, False)
    hinge = np.abs(g[0][:, 7:] - ref[0][:, 7:]).max()
    root = np.abs(g[0][:, :3] - ref[0][:, :3]).max()
    lerr = np.abs(g[3] - ref[3]).max()
    print(f"whole body tendon 200 steps: max hinge error {hinge:.2e} rad, root {root:.2e} m, "
          f"fibre {lerr:.2e} m, excursion {np.abs(ref[0][:, 7:] - q[:, 7:]).max():.2f} rad")
    assert hinge <= 1e-3 and root <= 1e-3 and lerr <= 1e-5


def test_tendon_failures_keep_the_state(chain):
    """An env whose fibre length is not finite is flagged and keeps its
    state; the others advance as they do alone."""
    m, gm, o = chain
    E, dt = 8, 2e-3
    q, qd, act, lm = _initial(m, o, synth.chain_initial_state, E)
    q, qd, act, lm = (v.astype(np.float32) for v in (q, qd, act, lm))
    lm_bad = lm.copy()
    lm_bad[3, 5] = np.nan
    us = [synth.excitation_iid(3, E, m["n_mus"], t) for t in range(4)]
    g = _gpu_steps(gm, q, qd, act, lm_bad, us, dt, False)
    ok = _gpu_steps(gm, q, qd, act, lm, us, dt, False)
    assert g[4][3] & ms.MS_ST_NONFINITE and (np.delete(g[4], 3) == 0).all()
    for i, x0 in enumerate((q, qd, act)):
        assert np.array_equal(g[i][3], x0[3])
        assert np.array_equal(np.delete(g[i], 3, axis=0), np.delete(ok[i], 3, axis=0))
    assert np.isnan(g[3][3, 5]) and np.array_equal(np.delete(g[3][3], 5), np.delete(lm_bad[3], 5))


def test_tendon_argument_errors(chain):
    """Invalid tendon arguments return MS_E_ARG before any launch."""
    m, gm, o = chain
    E = 4
    q, qd, act, lm = _initial(m, o, synth.chain_initial_state, E)
    a = [_t(q), _t(qd), _t(act), _t(lm)]
    ref = [v.clone() for v in a]
    st = torch.zeros(E, dtype=torch.int32, device=DEV)
    bad = {
        "eps0 = 0": dict(eps0=0.0),
        "beta = 0": dict(beta=0.0),
        "beta NaN": dict(beta=float("nan")),
        "eps0 inf": dict(eps0=float("inf")),
        "beta below 1.82 dt v_max": dict(beta=0.036),
    }
    for name, kw in bad.items():
        with pytest.raises(ms.MsError) as ei:
            gm.rollout_tendon(*a, st, 3, 2e-3, False, kind=ms.EXC_IID, seed=1, **kw)
        assert ei.value.code == -1, name
    with pytest.raises(ms.MsError):
        gm.rollout_tendon(a[0], a[1], a[2], None, st, 3, 2e-3, False, kind=ms.EXC_IID, seed=1)
    slack0 = ms.Model(models.mixed_chain() | {"l_slack": np.zeros(5, np.float32)})
    with pytest.raises(ms.MsError) as ei:
        slack0.rollout_tendon(_t(np.zeros((E, 5))), _t(np.zeros((E, 5))), _t(np.zeros((E, 5))),
                              _t(np.full((E, 5), 0.1)), st, 1, 2e-3, False, kind=ms.EXC_IID)
    assert ei.value.code == -1
    torch.cuda.synchronize()
    for x, y in zip(a, ref):
        assert torch.equal(x, y)


@pytest.mark.parametrize("which", ["chain", "human"])
def test_tendon_records_observables(which, chain, human):
    """A recorded tendon step advances the state bitwise as an unrecorded one
    and writes the oracle's stage values: the activation and the fibre length
    / l_opt at the step's start to float32 resolution (1e-6); the force of
    the right-hand side and the balancing fibre velocity within 4 times the
    oracle's spread under 4-ulp moves of the fibre lengths, or 1e-5 of the
    block's largest value; power |force Ldot|."""
    m, gm, o = chain if which == "chain" else human
    init = synth.chain_initial_state if which == "chain" else synth.human_initial_state
    dt, E = (2e-3, 8) if which == "chain" else (1e-3, 6)
    nm = m["n_mus"]
    q, qd, act, lm = _warm(m, o, init, E, 20, dt, False)
    u = synth.excitation_iid(7, E, nm, 0)
    obs = {k: torch.zeros(1, E, nm, device=DEV) for k in ("act", "force", "lm", "vm", "power")}
    nap = torch.zeros(E, dtype=torch.int32, device=DEV)
    a = [_t(q), _t(qd), _t(act), _t(lm)]
    st = torch.zeros(E, dtype=torch.int32, device=DEV)
    gm.rollout_tendon(*a, st, 1, dt, False, eps0=EPS0, beta=BETA, kind=ms.EXC_ARRAY,
                      u=_t(u[None]), every=1, obs=obs, n_applied=nap)
    torch.cuda.synchronize()
    plain = _gpu_steps(gm, q, qd, act, lm, [u], dt, False)
    for x, y in zip(a, plain[:4]):
        assert np.array_equal(x.cpu().numpy(), y)
    assert (st.cpu().numpy() == 0).all() and (nap.cpu().numpy() == 1).all()
    g = {k: v[0].cpu().numpy() for k, v in obs.items()}
    d64 = [v.astype(np.float64) for v in (q, qd, act, lm)]
    L = np.stack([o.geometry(d64[0][e], d64[1][e])[0] for e in range(E)])
    ulp = np.spacing(L.astype(np.float32)).astype(np.float64)
    rng = np.random.default_rng(8)
    for e in range(E):
        S = o.step_tendon(dt, d64[0][e], d64[1][e], d64[2][e], d64[3][e], u[e], EPS0, BETA,
                          contact=False, stages=True)[5]
        spread = {"F": 0.0, "vm": 0.0}
        for _ in range(3):
            lp = d64[3][e] + 4 * ulp[e] * rng.choice([-1.0, 1.0], size=nm)
            P = o.step_tendon(dt, d64[0][e], d64[1][e], d64[2][e], lp, u[e], EPS0, BETA,
                              contact=False, stages=True)[5]
            for k in spread:
                spread[k] = max(spread[k], np.abs(P[k] - S[k]).max())
        np.testing.assert_allclose(g["act"][e], S["act"], rtol=0, atol=1e-6)
        np.testing.assert_allclose(g["lm"][e], S["lm"], rtol=0, atol=1e-6 * max(np.abs(S["lm"]).max(), 1))
        for gk, sk in (("force", "F"), ("vm", "vm")):
            tol = max(4 * spread[sk], 1e-5 * max(np.abs(S[sk]).max(), 1.0))
            assert np.abs(g[gk][e] - S[sk]).max() <= tol, (gk, e)
        np.testing.assert_allclose(g["power"][e], np.abs(g["force"][e] * S["Ldot"]),
                                   rtol=1e-4, atol=1e-4 * np.abs(g["power"][e]).max())
