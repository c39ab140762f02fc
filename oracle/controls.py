"""FP32-resolvability controls of a free run (TEST INFRASTRUCTURE).

A whole-body trajectory with ground contact crosses discrete events (contact
onset, stick-slip). Where such an event falls at a time that perturbations at
float32 resolution shift, the trajectory has no unique float32 answer. These
controls measure that with the FP64 oracle alone, before any GPU result is
seen:

* rounding control: the oracle stepped with its state rounded to float32
  after every step (no other perturbation);
* event probe: the same with the generalised velocity also perturbed by a
  relative Gaussian of standard deviation PROBE_NOISE per step, PROBE_DRAWS
  seeded draws. PROBE_NOISE is ten times below the per-step bound of 1e-5 and
  of the order of the per-step error an FP32 step with an FP64 mass matrix
  makes on contact-free states.

An env is excluded from the free-run bound when the rounding control moves
its hinges by more than ROUND_EXCLUDE rad, or the probe by more than
PROBE_EXCLUDE rad. At most MAX_EXCLUDED_FRAC of the envs may be excluded.
These constants are fixed here, independently of any GPU run.
"""
from __future__ import annotations

import numpy as np

ROUND_EXCLUDE = 1e-4
PROBE_NOISE = 1e-6
PROBE_DRAWS = 4
PROBE_EXCLUDE = 1e-3
MAX_EXCLUDED_FRAC = 6 / 64


def _hinge_dev(qa, qb):
    return np.abs(qa[:, 7:] - qb[:, 7:]).max(axis=1)


def controlled_run(o, dt, q, qd, act, u, contact, noise=0.0, draws=1, seed=2024, ref=None):
    """Per-env max hinge deviation of the float32-rounded oracle (optionally
    with per-step relative velocity noise; max over draws) from the plain
    FP64 rollout (ref = its (final q, status) if already computed). q, qd,
    act: (E, .) float32 start states; u (T, E, n_mus)."""
    if ref is None:
        qo, _, _, so = o.rollout(dt, q, qd, act, u, contact=contact)
    else:
        qo, so = ref
    rng = np.random.default_rng(seed)
    dev = np.zeros(len(q))
    for _ in range(draws if noise > 0 else 1):
        qc, qdc, ac = q.copy(), qd.copy(), act.copy()
        for t in range(u.shape[0]):
            qc, qdc, ac, _ = o.rollout(dt, qc, qdc, ac, u[t:t + 1], contact=contact)
            if noise > 0:
                qdc = qdc * (1.0 + noise * rng.standard_normal(qdc.shape))
            qc, qdc, ac = (v.astype(np.float32) for v in (qc, qdc, ac))
        dev = np.maximum(dev, _hinge_dev(qc, qo))
    return dev, qo, so


def exclusions(o, dt, q, qd, act, u, contact=True):
    """Both controls and the excluded-env mask. Returns (excluded, rounding
    spread, probe spread, FP64 final q, FP64 status)."""
    r_dev, qo, so = controlled_run(o, dt, q, qd, act, u, contact)
    p_dev, _, _ = controlled_run(o, dt, q, qd, act, u, contact, noise=PROBE_NOISE,
                                 draws=PROBE_DRAWS, ref=(qo, so))
    excluded = (r_dev > ROUND_EXCLUDE) | (p_dev > PROBE_EXCLUDE)
    return excluded, r_dev, p_dev, qo, so
