"""FP64 oracle of the policy-driven rollout's inputs and outputs -- TEST
INFRASTRUCTURE (only the test-suite, the smoke check and the benchmark's
CPU-baseline leg use it).

Observation (paper, Methods, "Observation space": generalised position and
velocity plus reference targets; the paper's reference motion is replaced by
synthetic targets) and action (Methods, "Action space": one excitation in
[0, 1] per muscle), written from their definitions:

* position block: the generalised coordinates, a free root's unit
  quaternion (w, x, y, z) replaced by its rotation vector theta n with
  theta = 2 atan2(|v|, w) on the w >= 0 representative;
* velocity block: the generalised velocities;
* reference block: r_k(t) = sum_j A_kj sin(2 pi f_kj t + phi_kj);
* action: the sigmoid of the network output (mlp_forward with the GPU's
  bfloat16 rounding points).
"""
from __future__ import annotations

import numpy as np

from .oracle import mlp_forward


def quat_to_rotvec(xi):
    """Rotation vector of unit quaternions xi[..., 4] = (w, x, y, z)."""
    xi = np.asarray(xi, dtype=np.float64)
    sgn = np.where(xi[..., :1] < 0, -1.0, 1.0)
    xi = xi * sgn
    v = xi[..., 1:]
    s = np.linalg.norm(v, axis=-1, keepdims=True)
    theta = 2.0 * np.arctan2(s, xi[..., :1])
    scale = np.where(s > 1e-12, theta / np.where(s > 1e-12, s, 1.0), 2.0)
    return v * scale


def reference_targets(t, amp, freq, phase):
    """r[e, k] = sum_j amp[e,k,j] sin(2 pi freq[e,k,j] t + phase[e,k,j])."""
    amp, freq, phase = (np.asarray(a, dtype=np.float64) for a in (amp, freq, phase))
    return (amp * np.sin(2.0 * np.pi * freq * t + phase)).sum(axis=-1)


def policy_obs(model, q, qd, t, amp, freq, phase):
    """Observations [E][2 nv + n_ref] of states q[E][nq], qd[E][nv] at time t."""
    q = np.asarray(q, dtype=np.float64)
    qd = np.asarray(qd, dtype=np.float64)
    if model["jtype"][0] == 2:
        pos = np.concatenate([q[:, :3], quat_to_rotvec(q[:, 3:7]), q[:, 7:]], axis=1)
    else:
        pos = q
    return np.concatenate([pos, qd, reference_targets(t, amp, freq, phase)], axis=1)


def policy_act(params_in_out, obs, n_in):
    """Excitations sigmoid(net(obs)) with params (W1, b1, W2, b2, W3, b3),
    W[in][out], obs zero-padded to n_in inputs."""
    x = np.zeros((obs.shape[0], n_in))
    x[:, :obs.shape[1]] = obs
    y = mlp_forward(params_in_out, x, bf16=True)
    return 1.0 / (1.0 + np.exp(-y))
