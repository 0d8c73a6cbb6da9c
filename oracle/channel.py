"""Spherical-wave channel entries and the exact multiuser Gram G = H^H H.

Channel models
  PNUSW (paper eq. (3)):  h_i(m) = sqrt(beta0) e^{-j 2 pi r_im / lambda} / r_im * sqrt(x_i / r_im)
                          where x_i / r_im is the sine of the incidence angle; for 3-D users
                          x_i is the distance from the array line (ULA) or plane (UPA).
  FREESPACE:              h_i(m) = lambda / (4 pi r_im) e^{-j 2 pi r_im / lambda}
                          (the free-space model of the benchmark workloads).

Exact Gram (Sec. III, the inner products the paper wants to avoid, Sec. V-B):
  G_ij = sum_m conj(h_i(m)) h_j(m),  received power P_i = P G_ii,
  correlation rho_ij = G_ij / sqrt(G_ii G_jj).

Everything is FP64 and direct: the phase 2 pi r / lambda is formed in FP64 and
passed to ``numpy.exp`` without any range reduction.

Pins (tests/test_oracle_channel.py): far-field Dirichlet kernel, diagonal vs
the eq. (4) midpoint integral, large-N convergence to the eq. (6) phase and
magnitude, Hermitian / PSD / |rho| <= 1, mirror and permutation symmetry.
"""
from __future__ import annotations

import numpy as np

from workloads import AMP_FREESPACE, AMP_PNUSW, ArraySpec

from .geometry import element_positions, perpendicular_distance


def distances(arr: ArraySpec, users: np.ndarray) -> np.ndarray:
    """[N, K] element-to-user distances r_{k,n}."""
    e = element_positions(arr)
    u = np.asarray(users, np.float64)
    d = e[:, None, :] - u[None, :, :]
    return np.sqrt(np.sum(d * d, axis=-1))


def amplitudes(arr: ArraySpec, users: np.ndarray, r: np.ndarray) -> np.ndarray:
    """[N, K] real channel amplitudes |h_k(n)| for the array's amplitude model."""
    if arr.amp_model == AMP_FREESPACE:
        return arr.wavelength / (4.0 * np.pi * r)
    assert arr.amp_model == AMP_PNUSW
    xp = perpendicular_distance(arr, users)[None, :]
    return np.sqrt(arr.beta0) / r * np.sqrt(xp / r)


def channel_matrix(arr: ArraySpec, users: np.ndarray) -> np.ndarray:
    """H in C^{N x K}: column k is h_k of eq. (2), entries per eq. (3) / free space."""
    r = distances(arr, users)
    a = amplitudes(arr, users, r)
    return a * np.exp(-1j * (2.0 * np.pi / arr.wavelength) * r)


def gram_exact(arr: ArraySpec, users: np.ndarray, chunk: int = 16384) -> np.ndarray:
    """G = H^H H (K x K complex128), summed over element chunks to bound memory."""
    users = np.asarray(users, np.float64)
    k = users.shape[0]
    e_all = element_positions(arr)
    g = np.zeros((k, k), np.complex128)
    for s in range(0, e_all.shape[0], chunk):
        e = e_all[s:s + chunk]
        d = e[:, None, :] - users[None, :, :]
        r = np.sqrt(np.sum(d * d, axis=-1))
        a = amplitudes(arr, users, r)
        h = a * np.exp(-1j * (2.0 * np.pi / arr.wavelength) * r)
        g += h.conj().T @ h
    return g


def gram_exact_batch(arr: ArraySpec, drops, idx=None) -> list:
    """Exact Gram of each drop (list of K_d x K_d arrays), N taken per drop."""
    out = []
    for d in (range(drops.n_drops) if idx is None else idx):
        a = arr.with_n(int(drops.n_elems[d])) if arr.geometry == 0 else arr
        out.append(gram_exact(a, drops.users_of(d)))
    return out


def correlation(g: np.ndarray) -> np.ndarray:
    """rho_ij = G_ij / sqrt(G_ii G_jj) (Sec. III definition)."""
    dg = np.sqrt(np.real(np.diag(g)))
    return g / np.outer(dg, dg)


def normwise_error(g_test: np.ndarray, g_ref: np.ndarray) -> float:
    """max_ij |dG_ij| / sqrt(G_ii G_jj) with the reference diagonal."""
    dg = np.sqrt(np.abs(np.real(np.diag(g_ref))))
    return float(np.max(np.abs(g_test - g_ref) / np.outer(dg, dg)))
