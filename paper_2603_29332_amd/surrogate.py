"""Training and evaluation of the learned muscle-geometry surrogate.

Orchestration only: pose sampling, exact labels, forward, backward and Adam
all run in libms kernels (ms_surrogate_* and ms_geometry). Poses are drawn
uniformly inside the model's pose-domain box by a counter hash, so sample id
i of a seed is reproducible and labels are regenerated on the fly rather
than stored. Targets are standardised per output with statistics of a
separate labelled sample.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import ms


def _labels(gm, q, L, r):
    gm.geometry(q, L, r)


def output_stats(gm: ms.Model, s: ms.Surrogate, n: int = 8192, seed: int = 40):
    """Per-output mean and std over n sampled poses (empty moment-arm slots:
    mean 0, std 1)."""
    import torch
    dev = "cuda"
    q = torch.zeros(n, gm.nq, device=dev)
    L = torch.zeros(n, gm.n_mus, device=dev)
    r = torch.zeros(n, gm.n_mus, 3, device=dev)
    s.sample(q, seed, 0)
    _labels(gm, q, L, r)
    torch.cuda.synchronize()
    y = np.concatenate([L.cpu().numpy(), r.cpu().numpy().reshape(n, -1)], axis=1).astype(np.float64)
    mean = y.mean(0)
    std = y.std(0)
    spans = gm.spans().reshape(-1)
    empty = np.r_[np.zeros(gm.n_mus, bool), spans < 0]
    mean[empty] = 0.0
    std[empty] = 1.0
    std = np.maximum(std, 1e-6)
    return mean.astype(np.float32), std.astype(np.float32)


def train(gm: ms.Model, s: ms.Surrogate, n_samples: int = 10_000_000, batch: int = 8192,
          epochs: float = 1.0, lr0: float = 1e-2, lr1: float = 1e-5, seed: int = 41,
          log_every: int = 0, stream=None):
    """Adam with a cosine learning-rate decay from lr0 to lr1 over
    epochs * n_samples samples (sample ids cycle through 0..n_samples-1).
    Returns the per-iteration loss curve (float32 numpy) and the seconds."""
    import torch
    dev = "cuda"
    iters = max(1, int(round(epochs * n_samples / batch)))
    q = torch.zeros(batch, gm.nq, device=dev)
    L = torch.zeros(batch, gm.n_mus, device=dev)
    r = torch.zeros(batch, gm.n_mus, 3, device=dev)
    losses = torch.zeros(iters, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(iters):
        offset = (it * batch) % n_samples
        s.sample(q, seed, offset, stream=stream)
        gm.geometry(q, L, r, stream=stream)
        lr = lr1 + 0.5 * (lr0 - lr1) * (1.0 + math.cos(math.pi * it / iters))
        s.train_step(q, L, r, lr, it + 1, loss=losses[it:it + 1], stream=stream)
        if log_every and (it % log_every == 0 or it == iters - 1):
            torch.cuda.synchronize()
            print(f"  surrogate iter {it}/{iters} loss {losses[it].item():.3e} lr {lr:.2e}",
                  flush=True)
    torch.cuda.synchronize()
    return losses.cpu().numpy(), time.perf_counter() - t0


def evaluate(gm: ms.Model, s: ms.Surrogate, n: int = 100_000, seed: int = 43, chunk: int = 8192):
    """Errors of the network against exact geometry on n held-out poses:
    max and 99th percentile of |L_hat - L| (m) and |r_hat - r| (m)."""
    import torch
    dev = "cuda"
    errL, errR = [], []
    spans = gm.spans()
    have = spans >= 0
    for o in range(0, n, chunk):
        k = min(chunk, n - o)
        q = torch.zeros(k, gm.nq, device=dev)
        L = torch.zeros(k, gm.n_mus, device=dev)
        r = torch.zeros(k, gm.n_mus, 3, device=dev)
        Lh = torch.zeros_like(L)
        rh = torch.zeros_like(r)
        s.sample(q, seed, o)
        gm.geometry(q, L, r)
        s.forward(q, Lh, rh)
        torch.cuda.synchronize()
        errL.append(np.abs(Lh.cpu().numpy() - L.cpu().numpy()).max(axis=1))
        dr = np.abs(rh.cpu().numpy() - r.cpu().numpy())
        errR.append(np.where(have[None], dr, 0.0).max(axis=(1, 2)))
    eL = np.concatenate(errL)
    eR = np.concatenate(errR)
    return {"poses": n, "L_max_m": float(eL.max()), "L_p99_m": float(np.percentile(eL, 99)),
            "L_median_m": float(np.median(eL)), "r_max_m": float(eR.max()),
            "r_p99_m": float(np.percentile(eR, 99))}
