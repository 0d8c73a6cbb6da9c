"""Training and use of the learned closed-form correction.

Sequences library calls only (every computation is a kernel of libxlmimo):
exact FP32H Grams and closed-form Grams (variant GATED_QUAD, the learned form's base)
of training drops give per-pair
inputs and targets (xlmimo_mlp_pair_inputs); Adam steps run on contiguous
slices of the pair set (xlmimo_mlp_train_step).  Drops are generated in random
order, so a slice mixes many geometries without any gather.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import xlmimo as X


def init_params(width: int, depth: int, rng: np.random.Generator, log_var0: float) -> np.ndarray:
    """He-normal weights, zero biases; the output layer is scaled by 1e-2, its end-term
    coefficients start at 1 (the analytic end correction) and its log-variance bias at
    log_var0."""
    dims = [X.MLP_IN] + [width] * depth + [X.MLP_OUT]
    parts = []
    for li in range(len(dims) - 1):
        fan_in, fan_out = dims[li], dims[li + 1]
        w = rng.normal(0.0, math.sqrt(2.0 / fan_in), size=(fan_out, fan_in))
        b = np.zeros(fan_out)
        if li == len(dims) - 2:
            w *= 1e-2
            b[0] = 1.0   # c_top = 1
            b[2] = 1.0   # c_bot = 1
            b[6] = log_var0
        parts += [w.ravel(), b]
    return np.concatenate(parts).astype(np.float32)


def pair_set(ctx: X.Context, mlp: X.MLP, arr, drops, with_targets: bool = True):
    """Pair inputs (and targets rho_exact - rho~) of every drop; also returns the batch and Grams."""
    b = X.Batch(drops)
    g_cf, _ = ctx.gram_closedform(arr, b, X.CF_GATED_QUAD)
    g_ex = ctx.gram_exact(arr, b, X.FP32H) if with_targets else None
    return mlp.pair_inputs(arr, b, g_cf, g_ex), b, g_cf, g_ex


def train(mlp: X.MLP, data: X.PairInputs, steps: int, batch: int = 8192, lr_max: float = 2e-3,
          lr_min: float = 2e-5, log_every: int = 100):
    """Adam with a cosine learning-rate schedule over `steps` slices of `batch` pairs."""
    n = data.n
    n_batches = max(1, n // batch)
    loss = torch.empty(1, dtype=torch.float64, device=data.aux.device)
    history = []
    t0 = time.perf_counter()
    for s in range(steps):
        lr = lr_min + 0.5 * (lr_max - lr_min) * (1.0 + math.cos(math.pi * s / max(steps - 1, 1)))
        i = s % n_batches
        mlp.train_step(data.slice(i * batch, (i + 1) * batch), lr, loss)
        if (s + 1) % log_every == 0 or s == steps - 1:
            history.append((s + 1, float(loss.item())))
    torch.cuda.synchronize()
    return history, time.perf_counter() - t0
