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
    """He-normal weights, zero biases; the output layer is scaled by 1e-2 and its
    log-variance bias starts at log_var0.  Zero coefficient outputs are the analytic end
    correction (the kernels add its coefficients to the network's)."""
    dims = [X.MLP_IN] + [width] * depth + [X.MLP_OUT]
    parts = []
    for li in range(len(dims) - 1):
        fan_in, fan_out = dims[li], dims[li + 1]
        w = rng.normal(0.0, math.sqrt(2.0 / fan_in), size=(fan_out, fan_in))
        b = np.zeros(fan_out)
        if li == len(dims) - 2:
            w *= 1e-2
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
    """Adam with a cosine learning-rate schedule over `steps` slices of `batch` pairs (one
    library call enqueues every step)."""
    i = np.arange(steps, dtype=np.float64)
    lr = lr_min + 0.5 * (lr_max - lr_min) * (1.0 + np.cos(np.pi * i / max(steps - 1, 1)))
    loss = torch.empty(max(steps, 1), dtype=torch.float64, device=data.aux.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mlp.train(data, batch, lr.astype(np.float32), loss)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    lh = loss.cpu().numpy()
    history = [(s + 1, float(lh[s])) for s in range(steps) if (s + 1) % log_every == 0 or s == steps - 1]
    return history, secs


def constant_network(ctx: X.Context, width: int, depth: int, coeffs, log_var: float = -100.0) -> X.MLP:
    """A network whose output is the constant (coeffs, log_var) (zero weights, output bias
    only): coefficient outputs (0, 0, 0, 0, 0, 0) give the analytic end correction,
    (-1, 0, -1, 0, 0, 0) the base closed form alone."""
    m = X.MLP(ctx, width, depth)
    p = np.zeros(m.n_params, np.float32)
    p[-X.MLP_OUT:] = list(coeffs) + [log_var]
    m.set_params(p)
    return m


def drop_log_var(mlp: X.MLP, pi: X.PairInputs, n_drops: int) -> torch.Tensor:
    """Largest predicted log-variance over each drop's pairs (the quantity the fallback gate tests)."""
    out = mlp.forward(pi)
    lv = torch.full((n_drops,), -float("inf"), dtype=torch.float32, device=out.device)
    return lv.scatter_reduce(0, pi.pmap[:, 0].long(), out[:, 6], reduce="amax")


def calibrate_gate(ctx: X.Context, mlp: X.MLP, arr, drops, n_list, rho: torch.Tensor, target: float = 2.5e-4,
                   schemes: int = X.ZF | X.MMSE, min_keep: float = 0.9):
    """Fallback thresholds per antenna count, judged by the exact FP64 Gram on held-out drops.

    For each N the drops are ordered by their largest predicted log-variance; the threshold
    is the largest one whose kept drops all have a sum-rate error (relative, worst over the
    SNRs and schemes) of at most ``target`` with the network applied, or -inf when even
    the most certain drop misses it.  A threshold that keeps fewer than ``min_keep`` of the
    drops is set to -inf as well: where many drops miss the target, the predicted variance
    has not shown that it separates the good ones from the bad on new drops, and the closed
    form and the network would cost more than the exact kernel they spare (a batch whose
    every drop falls back skips them).  With a quarter as the bound, one of 1000 new drops at
    N = 256 kept by the gate missed 1e-3; with a half, after a retraining that left 51 % of the
    calibration drops at N = 256 within the target, one of 10^4 new drops missed it at 9.7e-3.
    Where the network is used (N >= 4096 on the sweep law) every calibration drop is within it.
    Returns (thresholds, per-N statistics)."""
    b = X.Batch(drops)
    thr, stats = [], []
    for n in n_list:
        a = arr.with_n(n)
        bn = X.Batch(drops.with_n(n), pos=b.pos)
        g64 = ctx.gram_exact(a, bn, X.FP64)
        gcf, _ = ctx.gram_closedform(a, bn, X.CF_GATED_QUAD)
        lv = drop_log_var(mlp, mlp.pair_inputs(a, bn, gcf), bn.n_drops)
        gml, _ = ctx.gram_closedform_mlp(a, bn, mlp, X.CF_GATED_QUAD, log_var_max=float("inf"))
        r64, _ = ctx.sumrate(bn, g64, rho, schemes)
        rml, _ = ctx.sumrate(bn, gml, rho, schemes)
        err = torch.nan_to_num(torch.abs(rml / r64 - 1), nan=float("inf")).amax(dim=(1, 2))
        lv_s, order = torch.sort(lv.double())
        ok = torch.cummax(err[order], dim=0).values <= target
        k = int(ok.long().cumprod(0).sum())          # longest prefix within the target
        while 0 < k < len(lv_s) and lv_s[k] == lv_s[k - 1]:
            k -= 1                                   # a threshold cannot split equal log-variances
        within = k / len(lv_s)
        if within < min_keep:
            k = 0
        t = float(lv_s[k - 1]) if k > 0 else -float("inf")
        thr.append(t)
        stats.append({"n": int(n), "log_var_max": t, "kept_fraction": k / len(lv_s),
                      "within_target_fraction": within,
                      "kept_err_max": float(err[order[:k]].max()) if k > 0 else 0.0,
                      "err_max_all": float(err.max())})
    mlp.set_gate(list(n_list), thr)
    return thr, stats
