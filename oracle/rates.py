"""Linear-receiver rates and capacity from a Gram matrix.

The paper fixes the uplink model y = Hx + n with E[xx^H] = P I (eq. (1)), the
capacity log2 det(I + (P/sigma^2) H^H H) (eq. (9)) and the ZF equaliser
x^ = (H^H H)^{-1} H^H y (eq. (21)); it prints no SINR formulas.  The oracle
uses the textbook per-user SINRs of linear receivers, with per-user transmit
SNR rho_k = P_k / sigma^2, D = diag(rho) and A = D^{1/2} G D^{1/2}:

  ZF       SINR_k = rho_k / [G^{-1}]_kk
  MMSE     SINR_k = 1 / [(I + A)^{-1}]_kk - 1
  MRC      SINR_k = rho_k G_kk^2 / (sum_{j != k} rho_j |G_kj|^2 + G_kk)
  CAP      log2 det(I + A)                                     (eq. (9))
  mismatched modified ZF: filter W = G~^{-1} H^H on the true channel,
           B = G~^{-1} G,
           SINR_k = rho_k |B_kk|^2 / (sum_{j != k} rho_j |B_kj|^2 + [G~^{-1} G G~^{-1}]_kk)

Sum-rate = sum_k log2(1 + SINR_k).  All inverses and determinants are LAPACK
(numpy.linalg) in FP64.

Pins (tests/test_oracle_rates.py): K = 1 reduces to log2(1 + rho ||h||^2);
ZF SINR equals the projection form rho ||P_perp h_k||^2 and MMSE SINR the
whitened-interference form, both computed from H itself; ZF <= MMSE <= CAP
<= Hadamard bound (Appendix A) and CAP >= the Schur-Horn lower bound;
the mismatched rate with G~ = G equals ZF; MMSE -> ZF as SNR grows.
The tracked Cholesky factor: the 2 x 2 closed form, L L^H = A with L lower
and a real positive diagonal, log2 det against the Leibniz expansion of the
determinant (3 x 3) and against the capacity.
"""
from __future__ import annotations

import numpy as np

SCHEME_ZF = 1
SCHEME_MMSE = 2
SCHEME_MRC = 4
SCHEME_CAP = 8
SCHEME_MZF = 16      # nominal modified ZF: ZF formula evaluated on G~
SCHEME_MZF_MISMATCH = 32
SCHEME_CORR_GAP = 64    # Appendix A: -(1/K) log2 det R, the normalised Hadamard / Schur-Horn gap


def sinr_zf(g, rho):
    ginv = np.linalg.inv(g)
    return rho / np.real(np.diag(ginv))


def sinr_mmse(g, rho):
    s = np.sqrt(rho)
    a = s[:, None] * g * s[None, :]
    m = np.linalg.inv(np.eye(g.shape[0]) + a)
    return 1.0 / np.real(np.diag(m)) - 1.0


def sinr_mrc(g, rho):
    gd = np.real(np.diag(g))
    p = np.abs(g) ** 2 * rho[None, :]
    interf = p.sum(axis=1) - rho * gd ** 2
    return rho * gd ** 2 / (interf + gd)


def capacity(g, rho):
    s = np.sqrt(rho)
    a = s[:, None] * g * s[None, :]
    sign, logdet = np.linalg.slogdet(np.eye(g.shape[0]) + a)
    return logdet / np.log(2.0)


def sinr_mismatched(g_true, g_filter, rho):
    ginv = np.linalg.inv(g_filter)
    b = ginv @ g_true
    noise = np.real(np.diag(ginv @ g_true @ ginv))
    p = np.abs(b) ** 2 * rho[None, :]
    sig = rho * np.abs(np.diag(b)) ** 2
    interf = p.sum(axis=1) - sig
    return sig / (interf + noise)


def sum_rate(sinr):
    return float(np.sum(np.log2(1.0 + sinr)))


def corr_gap(g):
    """Appendix A, eq. (9): the largest normalised gap (U - L) / U between the Hadamard upper bound and
    the Schur-Horn lower bound of the capacity, -(1/K) log2 det R, with R the correlation matrix
    r_ij = G_ij / sqrt(G_ii G_jj).  Independent of the SNR."""
    d = np.sqrt(np.real(np.diag(g)))
    r = g / np.outer(d, d)
    sign, logdet = np.linalg.slogdet(r)
    return float(-logdet / np.log(2.0) / g.shape[0]) if sign > 0 else float("nan")


def factored_matrix(g, rho=None):
    """The matrix whose Cholesky factor the tracking path keeps: G itself (rho None) or the
    capacity matrix I + D^{1/2} G D^{1/2} of eq. (9) for one SNR row rho."""
    if rho is None:
        return np.array(g, dtype=np.complex128)
    s = np.sqrt(np.asarray(rho, dtype=np.float64))
    return np.eye(g.shape[0]) + s[:, None] * g * s[None, :]


def cholesky_factor(g, rho=None):
    """The Cholesky factor of factored_matrix(g, rho): the unique lower-triangular L with a real
    positive diagonal and L L^H = A (LAPACK).  A tracking update must reach it for the updated A."""
    return np.linalg.cholesky(factored_matrix(g, rho))


def log2det(g, rho=None):
    """log2 det of factored_matrix(g, rho) from its factor, 2 sum log2 L_kk; with rho it is the
    capacity of eq. (9)."""
    return float(2.0 * np.sum(np.log2(np.real(np.diag(cholesky_factor(g, rho))))))


def rates(g_true, rho, schemes=SCHEME_ZF | SCHEME_MMSE, g_filter=None):
    """Dict scheme -> sum-rate [bit/s/Hz] for one drop."""
    rho = np.asarray(rho, np.float64)
    out = {}
    if schemes & SCHEME_ZF:
        out[SCHEME_ZF] = sum_rate(sinr_zf(g_true, rho))
    if schemes & SCHEME_MMSE:
        out[SCHEME_MMSE] = sum_rate(sinr_mmse(g_true, rho))
    if schemes & SCHEME_MRC:
        out[SCHEME_MRC] = sum_rate(sinr_mrc(g_true, rho))
    if schemes & SCHEME_CAP:
        out[SCHEME_CAP] = capacity(g_true, rho)
    if schemes & SCHEME_MZF:
        out[SCHEME_MZF] = sum_rate(sinr_zf(g_filter, rho))
    if schemes & SCHEME_MZF_MISMATCH:
        out[SCHEME_MZF_MISMATCH] = sum_rate(sinr_mismatched(g_true, g_filter, rho))
    if schemes & SCHEME_CORR_GAP:
        out[SCHEME_CORR_GAP] = corr_gap(g_true)
    return out


def hadamard_bound(g, rho):
    """Appendix A upper bound: log2 prod(1 + a_i), a_i the diagonal of D^{1/2} G D^{1/2}."""
    return float(np.sum(np.log2(1.0 + rho * np.real(np.diag(g)))))


def schur_horn_bound(g, rho):
    """Appendix A lower bound: log2( det(R) prod(1 + a_i) ), R the correlation matrix."""
    dg = np.sqrt(np.real(np.diag(g)))
    r = g / np.outer(dg, dg)
    sign, logdet = np.linalg.slogdet(r)
    return float(logdet / np.log(2.0) + hadamard_bound(g, rho))
