"""SNR convention of the benchmark workloads and the paper's experiments.

Not a computation of the method: the rate entry points take per-user
rho_k = P_k / sigma^2 as an input.  Here a common transmit power is set so that
a broadside reference user at a stated distance sees the stated SNR through
its array gain G_ref, the convention of the paper's Sec. V (the received SNR
limit of a reference user):
  ULA: the N -> infinity limit of the diagonal, free space
       (lambda / 4 pi)^2 pi / (d x) (lambda / (8 pi x) at d = lambda / 2),
       PNUSW 2 beta0 / (d x) (eq. (5) at d = lambda / 2);
  UPA (no finite limit): the far-field value of the panel's own diagonal,
       N (lambda / (4 pi x))^2 (free space) or N beta0 / x^2.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

import workloads as W


def reference_gain(arr, ref_distance: float) -> float:
    """Array gain G_ref of a broadside reference user at ``ref_distance`` (module docstring)."""
    lam, d, x = arr.wavelength, arr.spacing, float(ref_distance)
    if arr.geometry == W.GEOM_ULA:
        if arr.amp_model == W.AMP_FREESPACE:
            return (lam / (4 * np.pi)) ** 2 * np.pi / (d * x)
        return 2.0 * arr.beta0 / (d * x)
    n = arr.n_y * arr.n_z
    if arr.amp_model == W.AMP_FREESPACE:
        return n * (lam / (4 * np.pi * x)) ** 2
    return n * arr.beta0 / (x * x)


def rho_host(arr, snr_db: Sequence[float], ref_distance: float, total_users: int) -> np.ndarray:
    """float64 [n_snr, total_users]: P / sigma^2 = 10^(SNR/10) / G_ref for every user."""
    g = reference_gain(arr, ref_distance)
    vals = np.array([10.0 ** (s / 10.0) / g for s in snr_db], np.float64)
    return np.ascontiguousarray(np.broadcast_to(vals[:, None], (len(vals), max(total_users, 1))))


def rho_for_snr(arr, snr_db: Sequence[float], ref_distance: float, total_users: int, device=0):
    """rho_host as a CUDA tensor on ``device`` (the rate entry points read it from the device)."""
    import torch
    return torch.as_tensor(rho_host(arr, snr_db, ref_distance, total_users), device=f"cuda:{device}")
