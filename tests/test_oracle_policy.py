"""Pins of the policy-observation oracle (CPU): closed forms of the rotation
vector and of the reference sinusoids, and the block layout."""
import math

import numpy as np

from oracle import policy_obs, quat_to_rotvec, reference_targets
from paper_2603_29332_amd import synth


def _quat(axis, angle):
    axis = np.asarray(axis, float) / np.linalg.norm(axis)
    return np.r_[math.cos(angle / 2), math.sin(angle / 2) * axis]


def test_rotation_vector_closed_form_and_double_cover():
    rng = np.random.default_rng(0)
    for _ in range(20):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        th = rng.uniform(0, math.pi)
        xi = _quat(n, th)
        assert np.allclose(quat_to_rotvec(xi), th * n, atol=1e-12)
        assert np.allclose(quat_to_rotvec(-xi), th * n, atol=1e-12)   # same rotation
    assert np.allclose(quat_to_rotvec([1.0, 0, 0, 0]), 0.0)
    # a rotation by more than pi is the shorter one the other way round
    xi = _quat([0, 0, 1], 1.5 * math.pi)
    assert np.allclose(quat_to_rotvec(xi), [0, 0, -0.5 * math.pi], atol=1e-12)


def test_reference_targets_single_sinusoid_period_and_bound():
    amp = np.zeros((1, 1, 3))
    freq = np.ones((1, 1, 3))
    phase = np.zeros((1, 1, 3))
    amp[0, 0, 0], freq[0, 0, 0], phase[0, 0, 0] = 0.2, 1.25, 0.3
    for t in (0.0, 0.13, 0.77):
        r0 = reference_targets(t, amp, freq, phase)[0, 0]
        r1 = reference_targets(t + 1 / 1.25, amp, freq, phase)[0, 0]
        assert abs(r0 - r1) < 1e-12
    # quarter period past the zero crossing is the amplitude
    t = (math.pi / 2 - 0.3) / (2 * math.pi * 1.25)
    assert abs(reference_targets(t, amp, freq, phase)[0, 0] - 0.2) < 1e-12
    a, f, p = synth.reference_params(52, 8, 140)
    r = reference_targets(0.37, a, f, p)
    assert (np.abs(r) <= a.sum(axis=-1) + 1e-12).all()
    assert (a >= 0).all() and (a <= 0.3).all() and (f >= 0.5).all() and (f <= 2.0).all()


def test_observation_layout():
    m = synth.human_model(2)
    q, qd, _ = synth.human_initial_state(m, 3)
    rng = np.random.default_rng(1)
    qd = rng.normal(size=qd.shape)
    q = q.astype(np.float64)
    q[:, 3:7] = [_quat([1, 2, 3], 0.4)] * 3
    a, f, p = synth.reference_params(52, 3, 140)
    obs = policy_obs(m, q, qd, 0.25, a, f, p)
    assert obs.shape == (3, 300)
    assert np.allclose(obs[:, :3], q[:, :3])
    assert np.allclose(obs[:, 3:6], 0.4 * np.array([1, 2, 3]) / math.sqrt(14))
    assert np.allclose(obs[:, 6:80], q[:, 7:])
    assert np.allclose(obs[:, 80:160], qd)
    assert np.allclose(obs[:, 160:], reference_targets(0.25, a, f, p))


def test_action_is_the_sigmoid_of_the_network_output():
    """Zero weights give excitations of exactly 0.5; a large output bias
    saturates them at 1 (positive) or 0 (negative), never the reverse."""
    from oracle import policy_act
    n_in, h, n_out = 16, 8, 5
    z = [np.zeros((n_in, h)), np.zeros(h), np.zeros((h, h)), np.zeros(h),
         np.zeros((h, n_out)), np.zeros(n_out)]
    obs = np.random.default_rng(1).normal(size=(3, 12))
    assert np.array_equal(policy_act(z, obs, n_in), np.full((3, n_out), 0.5))
    up = list(z)
    up[5] = np.full(n_out, 50.0)
    assert np.allclose(policy_act(up, obs, n_in), 1.0)
    down = list(z)
    down[5] = np.full(n_out, -50.0)
    assert np.all(policy_act(down, obs, n_in) < 1e-20)
