"""FP64 oracle of the control step around the physics -- TEST INFRASTRUCTURE
(only the test-suite, the smoke check and the benchmark's CPU-baseline leg
use it).

Written from the paper's definitions (Methods):
* "Observation space": generalised position and velocity, key-body
  positions and orientations, muscle activations, forces, normalised fibre
  lengths and velocities, reference joint targets and reference key-body
  positions and orientations. Readings taken here: a free root's unit
  quaternion enters as its rotation vector; an orientation as the first two
  columns of its rotation matrix; forces divided by F0; the muscle state is
  that of the previous control step's last substep; the reference pose keeps
  the env's own root with the hinges at their targets.
* "Reinforcement learning with flow-based exploration" (Eq. pi_ode): a base
  action from the Gaussian initial sampler, a0 = mu(s) + sigma xi, refined by
  the flow velocity field, a = a0 + integral over [0, 1] of psi(t, s, a(t)),
  integrated here by explicit Euler steps t_k = k dt as the paper's ODE
  refinement; the action space is [0, 1] per muscle.
* "Unified imitation environment" (Eq. tracking_r): r = -log(1 - D(Delta)),
  Delta the tracking error between simulated and reference joint angles and
  body positions.
* "Simulation parameters": several physics substeps per control step with
  the excitations held.

Every network is evaluated by the FP64 MLP oracle with the GPU's bfloat16
rounding points (mlp_forward). The standard normal draws follow the
published Box-Muller transform of two counter-based uniforms.
"""
from __future__ import annotations

import numpy as np

from .oracle import mlp_forward
from .policy import quat_to_rotvec

_M64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """SplitMix64 output function (Steele, Lea & Flood 2014)."""
    z = (x + 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def unit24(z: int) -> float:
    return float(z >> 40) * 2.0 ** -24


def ref_hinge(seed: int, env: int, h: int, t: float) -> float:
    """Reference target of hinge h of env `env` at time t: three sinusoids
    with amplitude 0.3 a, frequency 0.5 + 1.5 b Hz and phase 2 pi c drawn
    from SplitMix64 on (seed, env, 3 h + j)."""
    ke = splitmix64(seed ^ env)
    s = 0.0
    for j in range(3):
        key = splitmix64(ke ^ (3 * h + j))
        A = 0.3 * unit24(splitmix64(key ^ 0))
        f = 0.5 + 1.5 * unit24(splitmix64(key ^ 1))
        ph = 2.0 * np.pi * unit24(splitmix64(key ^ 2))
        s += A * np.sin(2.0 * np.pi * f * t + ph)
    return s


def normal(seed: int, env: int, step: int, m: int) -> float:
    """Standard normal draw of muscle m: Box-Muller on two 24-bit uniforms
    of one SplitMix64 output, offset by half a unit so that u1 > 0."""
    z = splitmix64(splitmix64(splitmix64(seed ^ env) ^ step) ^ m)
    u1 = ((z >> 40) + 0.5) * 2.0 ** -24
    u2 = (((z >> 16) & 0xFFFFFF) + 0.5) * 2.0 ** -24
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def hinge_coords(model):
    """q index of every hinge/slide coordinate, in node order."""
    out, qa = [], 0
    for i in range(model["n_node"]):
        if model["jtype"][i] == 2:
            qa += 7
            continue
        out.append(qa)
        qa += 1
    return np.array(out)


def reference_pose(model, q, env, t, seed):
    """The env's root with every hinge at its reference target."""
    qr = np.array(q, dtype=np.float64)
    for h, j in enumerate(hinge_coords(model)):
        qr[j] = ref_hinge(seed, env, h, t)
    return qr


def key_frames(o, q, keys):
    """World positions [n_key][3] and rotations [n_key][3][3] of key nodes."""
    R, p = o.fk(np.asarray(q, dtype=np.float64))
    return p[keys], R[keys]


def observation(model, o, q, qd, mstate_env, t, env, keys, ref_seed):
    """Observation of one env (see the module docstring for the order)."""
    q = np.asarray(q, dtype=np.float64)
    if model["jtype"][0] == 2:
        pos = np.concatenate([q[:3], quat_to_rotvec(q[3:7]), q[7:]])
    else:
        pos = q
    kp, kR = key_frames(o, q, keys)
    qr = reference_pose(model, q, env, t, ref_seed)
    rp, rR = key_frames(o, qr, keys)
    six = lambda R: np.concatenate([R[:, :, 0], R[:, :, 1]], axis=1).reshape(-1)
    act, F, lm, vm = (np.asarray(x, dtype=np.float64) for x in mstate_env)
    f0 = np.asarray(model["f0"], dtype=np.float64)
    return np.concatenate([pos, np.asarray(qd, dtype=np.float64), kp.reshape(-1), six(kR),
                           act, F / f0, lm, vm, qr[hinge_coords(model)], rp.reshape(-1), six(rR)])


def pad(x, n):
    y = np.zeros(n)
    y[:len(x)] = x
    return y


def sample_action(pi_params, flow_params, log_std, obs, n_in, n_at, n_mus, env, step,
                  noise_seed, flow_steps, flow_dt):
    """Initial sample a0 = mu + exp(log_std) xi, then flow_steps Euler steps
    a += flow_dt psi(t_k, s, a) on the flow network's input [s, a, t_k];
    returns (a0, clip(a, 0, 1))."""
    s = pad(obs, n_in)
    mu = mlp_forward(pi_params, s[None], bf16=True)[0]
    xi = np.array([normal(noise_seed, env, step, m) for m in range(n_mus)])
    a0 = mu + np.exp(np.asarray(log_std, dtype=np.float64)) * xi
    a = a0.copy()
    for k in range(flow_steps):
        x = np.concatenate([s, pad(np.r_[a, k * flow_dt], n_at)])
        a = a + flow_dt * mlp_forward(flow_params, x[None], bf16=True)[0]
    return a0, np.clip(a, 0.0, 1.0)


def tracking_error(model, o, q, env, t, keys, ref_seed):
    """[hinge coordinates - targets, key positions - reference key positions]."""
    qr = reference_pose(model, q, env, t, ref_seed)
    hc = hinge_coords(model)
    kp, _ = key_frames(o, q, keys)
    rp, _ = key_frames(o, qr, keys)
    return np.concatenate([np.asarray(q, dtype=np.float64)[hc] - qr[hc], (kp - rp).reshape(-1)])


def reward(disc_params, delta, n_din):
    """-log(1 - sigmoid(z)) with z the discriminator's output."""
    z = mlp_forward(disc_params, pad(delta, n_din)[None], bf16=True)[0, 0]
    return float(np.logaddexp(0.0, z))


def substeps(o, dt, q, qd, act, u, n_sub, contact):
    """n_sub oracle steps with u held; returns the state, status and the last
    substep's muscle state (act', F, l_m, v_m)."""
    st_all = 0
    last = None
    for k in range(n_sub):
        q, qd, act, st, S = o.step(dt, q, qd, act, u, contact=contact, stages=True)
        st_all |= st
        last = (S["act"], S["F"], S["lm"], S["vm"])
    return q, qd, act, st_all, last
