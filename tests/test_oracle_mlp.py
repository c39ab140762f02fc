"""Pins of the FP64 surrogate-network oracle: bfloat16 rounding, a
hand-computed forward pass, gradients against central differences, Adam's
first step in closed form."""
import math

import numpy as np

import oracle
from oracle import oracle as ora


def test_bf16_round_to_nearest_even():
    assert oracle.bf16(1.0) == 1.0
    assert oracle.bf16(1 + 2 ** -8) == 1.0                   # tie -> even
    assert oracle.bf16(1 + 3 * 2 ** -8) == 1 + 2 ** -6        # tie -> even (up)
    assert oracle.bf16(1 + 2 ** -8 + 2 ** -20) == 1 + 2 ** -7  # above the tie
    assert oracle.bf16(-2.5) == -2.5
    assert math.isinf(oracle.bf16(1e39))                        # float32 overflow
    assert math.isnan(oracle.bf16(float("nan")))


def _silu(z):
    return z / (1 + math.exp(-z))


def test_forward_by_hand():
    W1 = np.array([[0.5, -1.0], [2.0, 0.25]])
    b1 = np.array([0.1, -0.2])
    W2 = np.array([[1.0, 0.0], [-0.5, 1.5]])
    b2 = np.array([0.0, 0.3])
    W3 = np.array([[2.0], [-1.0]])
    b3 = np.array([0.5])
    x = np.array([[1.0, -0.5]])
    z1 = [1.0 * 0.5 - 0.5 * 2.0 + 0.1, 1.0 * -1.0 - 0.5 * 0.25 - 0.2]
    h1 = [_silu(z) for z in z1]
    z2 = [h1[0] * 1.0 + h1[1] * -0.5, h1[0] * 0.0 + h1[1] * 1.5 + 0.3]
    h2 = [_silu(z) for z in z2]
    y = h2[0] * 2.0 - h2[1] + 0.5
    out = oracle.mlp_forward((W1, b1, W2, b2, W3, b3), x, bf16=False)
    assert abs(out[0, 0] - y) < 1e-7   # float32-stored biases/weights are exact here


def _net(rng, n0=5, n1=7, n2=6, n3=4):
    return [rng.normal(size=(n0, n1)) * 0.5, rng.normal(size=n1) * 0.1,
            rng.normal(size=(n1, n2)) * 0.5, rng.normal(size=n2) * 0.1,
            rng.normal(size=(n2, n3)) * 0.5, rng.normal(size=n3) * 0.1]


def test_gradients_match_central_differences():
    rng = np.random.default_rng(0)
    P = [p.astype(np.float32) for p in _net(rng)]
    x = rng.normal(size=(9, 5)).astype(np.float32)
    t = rng.normal(size=(9, 4)).astype(np.float32)
    mask = (rng.uniform(size=(9, 4)) > 0.2).astype(np.float32)
    loss, g = oracle.mlp_grad(P, x, t, mask, bf16=False)
    h = 1e-3   # parameters are float32: perturb by an exactly representable step
    for k, p in enumerate(P):
        flat = p.reshape(-1)
        for idx in range(0, flat.size, max(1, flat.size // 6)):
            old = flat[idx]
            flat[idx] = old + np.float32(h)
            lp, _ = oracle.mlp_grad(P, x, t, mask, bf16=False)
            flat[idx] = old - np.float32(h)
            lm, _ = oracle.mlp_grad(P, x, t, mask, bf16=False)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[k].reshape(-1)[idx]) < 1e-6 + 1e-5 * abs(fd), (k, idx)


def test_masked_outputs_carry_no_gradient():
    rng = np.random.default_rng(1)
    P = [p.astype(np.float32) for p in _net(rng)]
    x = rng.normal(size=(4, 5)).astype(np.float32)
    t = rng.normal(size=(4, 4)).astype(np.float32)
    loss, g = oracle.mlp_grad(P, x, t, np.zeros((4, 4), np.float32), bf16=True)
    assert loss == 0.0 and all(np.abs(gi).max() == 0.0 for gi in g)


def test_bf16_gradients_close_to_exact():
    rng = np.random.default_rng(2)
    P = [p.astype(np.float32) for p in _net(rng, 16, 32, 32, 8)]
    x = rng.normal(size=(64, 16)).astype(np.float32)
    t = rng.normal(size=(64, 8)).astype(np.float32)
    _, g0 = oracle.mlp_grad(P, x, t, None, bf16=False)
    _, g1 = oracle.mlp_grad(P, x, t, None, bf16=True)
    for a, b in zip(g0, g1):
        assert np.abs(a - b).max() <= 3e-2 * np.abs(a).max()


def test_adam_first_step_and_bias_correction():
    w = np.array([1.0, -2.0, 0.0])
    m = np.zeros(3)
    v = np.zeros(3)
    g = np.array([0.5, -4.0, 0.0])
    oracle.adam(w, m, v, g, lr=0.1, step=1)
    # bias-corrected first step moves by lr * g / (|g| + eps)
    expect = np.array([1.0, -2.0, 0.0]) - 0.1 * g / (np.abs(g) + 1e-8)
    assert np.allclose(w, expect, rtol=0, atol=1e-12)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
    # second step with the same gradient: m_hat = g, v_hat = g^2 again
    oracle.adam(w, m, v, g, lr=0.1, step=2)
    assert np.allclose(w, expect - 0.1 * g / (np.abs(g) + 1e-8), atol=1e-12)
