"""Training of the learned muscle-geometry surrogate (argument passing only).

Pose sampling, exact labels, the output standardisation, forward, backward,
Adam and the cosine learning-rate schedule all run in libms
(ms_surrogate_train); this module only converts an epoch count into steps.
"""
from __future__ import annotations

import time

from . import ms


def train(s: ms.Surrogate, n_samples: int = 10_000_000, batch: int = 8192, epochs: float = 1.0,
          lr0: float = 1e-2, lr1: float = 1e-5, seed: int = 41, norm_samples: int = 8192,
          norm_seed: int = 40, stream=None):
    """Train for epochs * n_samples samples (sample ids cycle through
    0..n_samples-1), the output standardisation first from norm_samples
    poses. Returns the per-step loss (float32 numpy) and the seconds."""
    import torch
    iters = max(1, int(round(epochs * n_samples / batch)))
    losses = torch.zeros(iters, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.train(n_samples=n_samples, batch=batch, iters=iters, lr0=lr0, lr1=lr1, seed=seed,
            norm_samples=norm_samples, norm_seed=norm_seed, loss=losses, stream=stream)
    torch.cuda.synchronize()
    return losses.cpu().numpy(), time.perf_counter() - t0
