"""Pins of the oracle's rate formulas against forms computed from H itself
(projection, whitened interference, Sylvester determinant) and the bounds of
Appendix A."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import channel as ch
from oracle import rates as R


def _drop(n=24, k=5, seed=1, amp=W.AMP_FREESPACE):
    rng = np.random.default_rng(seed)
    arr = W.ula(n, W.LAMBDA_28GHZ, amp)
    r = rng.uniform(1.0, 6.0, k)
    th = rng.uniform(-1.0, 1.0, k)
    u = np.stack([r * np.cos(th), r * np.sin(th), np.zeros(k)], axis=-1)
    h = ch.channel_matrix(arr, u)
    g = h.conj().T @ h
    rho = rng.uniform(0.5, 2.0, k) * 10.0 / np.real(np.diag(g)).mean()
    return h, g, rho


def test_single_user_reduces_to_awgn():
    h, g, rho = _drop(k=1)
    want = math.log2(1 + rho[0] * np.linalg.norm(h) ** 2)
    out = R.rates(g, rho, R.SCHEME_ZF | R.SCHEME_MMSE | R.SCHEME_MRC | R.SCHEME_CAP)
    for v in out.values():
        assert v == pytest.approx(want, rel=1e-13)


def test_zf_equals_projection_form():
    # ZF SINR_k = rho_k || P_perp(H_{-k}) h_k ||^2, P_perp the projector orthogonal to the other users
    h, g, rho = _drop()
    s = R.sinr_zf(g, rho)
    for k in range(h.shape[1]):
        others = np.delete(h, k, axis=1)
        coef, *_ = np.linalg.lstsq(others, h[:, k], rcond=None)
        resid = h[:, k] - others @ coef
        assert s[k] == pytest.approx(rho[k] * np.linalg.norm(resid) ** 2, rel=1e-8)


def test_mmse_equals_whitened_form():
    # MMSE SINR_k = rho_k h_k^H (I + sum_{j != k} rho_j h_j h_j^H)^{-1} h_k   (sigma^2 = 1)
    h, g, rho = _drop()
    s = R.sinr_mmse(g, rho)
    n = h.shape[0]
    for k in range(h.shape[1]):
        c = np.eye(n, dtype=complex)
        for j in range(h.shape[1]):
            if j != k:
                c += rho[j] * np.outer(h[:, j], h[:, j].conj())
        want = rho[k] * np.real(h[:, k].conj() @ np.linalg.solve(c, h[:, k]))
        assert s[k] == pytest.approx(want, rel=1e-9)


def test_mrc_and_capacity_from_h():
    h, g, rho = _drop()
    s = R.sinr_mrc(g, rho)
    for k in range(h.shape[1]):
        w = h[:, k]
        sig = rho[k] * abs(w.conj() @ h[:, k]) ** 2
        interf = sum(rho[j] * abs(w.conj() @ h[:, j]) ** 2 for j in range(h.shape[1]) if j != k)
        assert s[k] == pytest.approx(sig / (interf + np.linalg.norm(w) ** 2), rel=1e-12)
    # eq. (9) via Sylvester: det(I_K + D^1/2 G D^1/2) = det(I_N + H D H^H)
    _, ld = np.linalg.slogdet(np.eye(h.shape[0]) + (h * rho) @ h.conj().T)
    assert R.capacity(g, rho) == pytest.approx(ld / math.log(2), rel=1e-12)


def test_mismatched_from_filter():
    h, g, rho = _drop(seed=4)
    rng = np.random.default_rng(5)
    e = rng.normal(size=g.shape) + 1j * rng.normal(size=g.shape)
    gt = g + 0.01 * np.abs(g).max() * (e + e.conj().T)   # a Hermitian filter Gram
    s = R.sinr_mismatched(g, gt, rho)
    w = np.linalg.inv(gt) @ h.conj().T                    # W = G~^{-1} H^H
    b = w @ h
    for k in range(h.shape[1]):
        sig = rho[k] * abs(b[k, k]) ** 2
        interf = sum(rho[j] * abs(b[k, j]) ** 2 for j in range(h.shape[1]) if j != k)
        assert s[k] == pytest.approx(sig / (interf + np.linalg.norm(w[k]) ** 2), rel=1e-9)
    # with the true Gram as the filter it is ZF
    assert np.allclose(R.sinr_mismatched(g, g, rho), R.sinr_zf(g, rho), rtol=1e-9)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_orderings_and_appendix_a_bounds(seed):
    h, g, rho = _drop(seed=seed, amp=W.AMP_PNUSW)
    zf, mm = R.sinr_zf(g, rho), R.sinr_mmse(g, rho)
    assert np.all(zf <= mm * (1 + 1e-12))
    cap = R.capacity(g, rho)
    assert R.sum_rate(mm) <= cap + 1e-12
    assert cap <= R.hadamard_bound(g, rho) + 1e-12
    assert cap >= R.schur_horn_bound(g, rho) - 1e-12


def test_mmse_tends_to_zf_at_high_snr():
    h, g, rho = _drop()
    big = rho * 1e10
    assert np.allclose(R.sinr_mmse(g, big), R.sinr_zf(g, big), rtol=1e-6)


def test_corr_gap_appendix_a():
    # -(1/K) log2 det R (Appendix A, eq. (9)): zero for orthogonal users; for two users
    # -1/2 log2(1 - |r12|^2); equal to the negative mean log2-eigenvalue of R (the paper's last form);
    # and equal to the normalised log-gap between the Hadamard and Schur-Horn bounds at a_i = 1 (0 dB)
    assert abs(R.corr_gap(np.diag([2.0, 5.0, 0.5]).astype(np.complex128))) < 1e-15   # sqrt rounding only
    g2 = np.array([[4.0, 0.6 - 0.8j], [0.6 + 0.8j, 1.0]])
    r12 = abs(g2[0, 1]) / np.sqrt(4.0 * 1.0)
    assert R.corr_gap(g2) == pytest.approx(-0.5 * np.log2(1 - r12 ** 2), rel=1e-14)
    for seed in (1, 2):
        h, g, rho = _drop(seed=seed, amp=W.AMP_PNUSW)
        d = np.sqrt(np.real(np.diag(g)))
        lam = np.linalg.eigvalsh(g / np.outer(d, d))
        assert R.corr_gap(g) == pytest.approx(-np.mean(np.log2(lam)), rel=1e-10)
        unit = 1.0 / np.real(np.diag(g))                      # a_i = rho_i G_ii = 1
        u, lo = R.hadamard_bound(g, unit), R.schur_horn_bound(g, unit)
        assert R.corr_gap(g) == pytest.approx((u - lo) / u, rel=1e-10)


def test_cholesky_factor_two_by_two_closed_form():
    # A = [[a, b], [conj b, c]]: L = [[sqrt a, 0], [conj(b) / sqrt a, sqrt(c - |b|^2 / a)]]
    a, b, c = 2.5, 0.7 - 1.1j, 3.0
    L = R.cholesky_factor(np.array([[a, b], [np.conj(b), c]]))
    want = np.array([[math.sqrt(a), 0.0], [np.conj(b) / math.sqrt(a), math.sqrt(c - abs(b) ** 2 / a)]])
    assert np.allclose(L, want, rtol=0, atol=1e-15)


def test_cholesky_factor_properties_and_log2det():
    h, g, rho = _drop(n=40, k=6, seed=4)
    for r in (None, rho):
        A = R.factored_matrix(g, r)
        L = R.cholesky_factor(g, r)
        assert np.array_equal(np.triu(L, 1), np.zeros_like(L))
        d = np.diag(L)
        assert np.all(np.abs(d.imag) == 0) and np.all(d.real > 0)
        assert np.abs(L @ L.conj().T - A).max() <= 1e-14 * np.abs(A).max()
    # with rho, log2 det is the capacity of eq. (9)
    assert R.log2det(g, rho) == pytest.approx(R.capacity(g, rho), rel=1e-13)


def test_log2det_against_leibniz_expansion():
    # 3 x 3 determinant by its permutation expansion, independent of any factorisation
    import itertools
    h, g, rho = _drop(n=30, k=3, seed=6)
    det = 0.0
    for perm in itertools.permutations(range(3)):
        sign = (-1) ** sum(perm[i] > perm[j] for i in range(3) for j in range(i + 1, 3))   # inversions
        det += sign * g[0, perm[0]] * g[1, perm[1]] * g[2, perm[2]]
    assert abs(det.imag) < 1e-12 * abs(det.real)
    assert R.log2det(g) == pytest.approx(math.log2(det.real), rel=1e-12)
