"""Pins of the oracle's channel model and exact Gram against results fixed by
the mathematics, not by re-running the oracle's own formula.

Each pin is chosen so that a plausible slip fails it:
  * element centring or spacing wrong      -> Dirichlet kernel, mirror symmetry
  * phase sign / conjugation / transpose   -> Dirichlet prefactor, eq. (6) phase
  * amplitude model wrong (sqrt dropped)   -> diagonal vs eq. (4) integral
  * UPA indexing wrong                     -> UPA(n_y, 1) == ULA, UPA(1, n_z) == rotated ULA
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import channel as ch
from oracle import closedform as cf
from oracle import geometry


def _users(pts):
    return np.array([[p[0], p[1], 0.0 if len(p) == 2 else p[2]] for p in pts], np.float64)


def test_single_element_rank_one():
    # N = 1: the only element sits at the origin, r_k = |p_k|, so
    # G_ij = a_i a_j exp(+j k (r_i - r_j)) (h ~ exp(-j k r), G = H^H H).
    lam = 0.0107
    arr = W.ula(1, lam)
    u = _users([(3.0, 4.0), (6.0, -8.0), (1.0, 0.0)])
    g = ch.gram_exact(arr, u)
    r = np.array([5.0, 10.0, 1.0])
    a = lam / (4 * math.pi * r)
    k = 2 * math.pi / lam
    want = np.outer(a, a) * np.exp(1j * k * (r[:, None] - r[None, :]))
    # phases k r ~ 6e3 rad carry FP64 rounding of ~1e-12 rad
    assert np.allclose(g, want, rtol=0, atol=1e-11 * np.abs(want).max())
    assert np.linalg.matrix_rank(g, tol=1e-12 * np.abs(g).max()) == 1


def test_far_field_dirichlet_kernel():
    # Users at r >> aperture^2/lambda: r_n = r - y_n sin(theta) + O(y_n^2 / r), so
    # rho_ij -> exp(j k (r_i - r_j)) sin(N psi / 2) / (N sin(psi / 2)),
    # psi = k delta (sin theta_j - sin theta_i), for a centred array.
    lam = W.LAMBDA_28GHZ
    n = 16
    arr = W.ula(n, lam)
    r0 = 1.0e5
    th = np.deg2rad([12.0, -20.0, 31.0])
    u = np.stack([r0 * np.cos(th), r0 * np.sin(th), np.zeros(3)], axis=-1)
    u[1] *= 1.0 + 3e-6   # make r_i - r_j non-zero so the prefactor phase matters
    rho = ch.correlation(ch.gram_exact(arr, u))
    k = 2 * math.pi / lam
    r = np.linalg.norm(u, axis=1)
    s = np.sin(th)
    for i in range(3):
        for j in range(3):
            psi = k * arr.spacing * (s[j] - s[i])
            dk = n if i == j else math.sin(n * psi / 2) / math.sin(psi / 2)
            want = np.exp(1j * k * (r[i] - r[j])) * dk / n
            # neglected curvature phase k y^2 / (2 r) <= 5.3e-6 rad at this size
            assert abs(rho[i, j] - want) < 2e-5, (i, j, rho[i, j], want)


@pytest.mark.parametrize("amp", [W.AMP_FREESPACE, W.AMP_PNUSW])
def test_invariants(amp):
    rng = np.random.default_rng(7)
    arr = W.ula(300, W.LAMBDA_28GHZ, amp)
    k = 6
    r = rng.uniform(2, 20, k)
    th = rng.uniform(-1.0, 1.0, k)
    u = np.stack([r * np.cos(th), r * np.sin(th), np.zeros(k)], axis=-1)
    g = ch.gram_exact(arr, u)
    # Hermitian with a real positive diagonal equal to sum |h|^2
    assert np.allclose(g, g.conj().T, rtol=0, atol=1e-15 * np.abs(g).max())
    h = ch.channel_matrix(arr, u)
    assert np.allclose(np.diag(g).real, np.sum(np.abs(h) ** 2, axis=0), rtol=1e-13)
    assert np.all(np.abs(np.diag(g).imag) < 1e-16 * np.abs(g).max())
    # positive definite for distinct users, K <= N; |rho| <= 1
    np.linalg.cholesky(g)
    rho = ch.correlation(g)
    assert np.all(np.abs(rho) <= 1 + 1e-12)
    # mirror y -> -y of every user leaves G unchanged (array symmetric about y = 0)
    um = u * np.array([1, -1, 1])
    assert np.allclose(ch.gram_exact(arr, um), g, rtol=1e-10, atol=1e-14 * np.abs(g).max())
    # permutation equivariance
    p = rng.permutation(k)
    assert np.allclose(ch.gram_exact(arr, u[p]), g[np.ix_(p, p)], rtol=1e-12, atol=0)
    # chunked accumulation equals a single product
    assert np.allclose(ch.gram_exact(arr, u, chunk=7), h.conj().T @ h, rtol=1e-12, atol=1e-15 * np.abs(g).max())


def test_elements_centred():
    arr = W.ula(5, 0.02)
    e = geometry.element_positions(arr)
    assert np.allclose(e[:, 1], [-0.02, -0.01, 0.0, 0.01, 0.02])
    arr = W.ula(4, 0.02)
    assert np.allclose(geometry.element_positions(arr)[:, 1], [-0.015, -0.005, 0.005, 0.015])


def test_upa_reduces_to_ula():
    lam = W.LAMBDA_100GHZ_UPA
    rng = np.random.default_rng(3)
    u = np.stack([rng.uniform(1, 5, 4), rng.uniform(-2, 2, 4), np.zeros(4)], axis=-1)
    ula = W.ArraySpec(W.GEOM_ULA, 64, 1, lam / 2, lam)
    upa_row = W.ArraySpec(W.GEOM_UPA, 64, 1, lam / 2, lam)
    assert np.allclose(ch.gram_exact(upa_row, u), ch.gram_exact(ula, u), rtol=1e-13, atol=0)
    # a 1 x n_z panel is a ULA along z: rotate the users y -> z
    upa_col = W.ArraySpec(W.GEOM_UPA, 1, 64, lam / 2, lam)
    ur = u[:, [0, 2, 1]]
    assert np.allclose(ch.gram_exact(upa_col, ur), ch.gram_exact(ula, u), rtol=1e-12, atol=0)


@pytest.mark.parametrize("n", [256, 4096, 65536])
def test_diagonal_matches_eq4_integral(n):
    # eq. (4) is the midpoint rule of the diagonal; its error is O(delta^2 f'') and
    # falls with n (measured 1e-8 at n = 256 in this geometry).
    lam = W.LAMBDA_100GHZ
    arr = W.ula(n, lam, W.AMP_PNUSW)
    u = _users([(1.5, 0.3), (7.0, -4.0)])
    g = ch.gram_exact(arr, u)
    want = cf.power_eq4(u[:, 0], u[:, 1], n, lam)
    assert np.allclose(np.diag(g).real, want, rtol=1e-6)


def test_large_m_converges_to_eq6():
    # eq. (6) is the stationary-phase value of rho; with the stationary point well
    # inside a long PNUSW array the exact correlation approaches it (normwise about
    # 2.6e-6 at M = 262144, lambda = 3 mm).  The phase part pins the
    # conjugation convention G = H^H H with h ~ exp(-j k r).
    lam = W.LAMBDA_100GHZ
    arr = W.ula(262144, lam, W.AMP_PNUSW)
    u = _users([(2.0, 0.5), (4.0, 1.7), (1.2, -0.8)])
    rho = ch.correlation(ch.gram_exact(arr, u))
    for i, j in [(0, 1), (1, 0), (0, 2), (2, 1)]:
        want = cf.rho_eq6(u[i, 0], u[i, 1], u[j, 0], u[j, 1], 262144, lam)
        # normwise (absolute on rho) error of the stationary-phase term ~ 3e-6 here
        assert abs(rho[i, j] - want) < 1e-5, (i, j, rho[i, j], want)
        assert abs(rho[i, j] - want) < 1e-3 * abs(want)
        assert abs(np.angle(rho[i, j] / want)) < 1e-2


def test_three_d_user_ula_rotation():
    # A ULA channel depends only on (sqrt(x^2 + z^2), y) (rotation about the array axis).
    arr = W.ula(128, 0.01, W.AMP_PNUSW)
    u2 = _users([(3.0, 0.4), (5.0, -1.0)])
    ang = 0.7
    u3 = np.array([[3.0 * math.cos(ang), 0.4, 3.0 * math.sin(ang)], [5.0, -1.0, 0.0]])
    assert np.allclose(ch.gram_exact(arr, u3), ch.gram_exact(arr, u2), rtol=1e-10, atol=0)
