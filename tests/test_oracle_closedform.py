"""Pins of the oracle's closed forms (eqs. (4)-(8), (22)-(23) and the derived
free-space / UPA forms) against quadrature, limits and the exact Gram."""
import math

import numpy as np
import pytest
from scipy import integrate

import workloads as W
from oracle import channel as ch
from oracle import closedform as cf


def _users(pts):
    return np.array([[p[0], p[1], 0.0 if len(p) == 2 else p[2]] for p in pts], np.float64)


@pytest.mark.parametrize("x,y,m", [(1.5, 0.0, 4096), (7.0, -3.0, 1000), (2.0, 5.0, 20000)])
def test_eq4_is_the_aperture_integral(x, y, m):
    # eq. (4)/P = (1/delta) int_{-L}^{L} beta0 x / (x^2 + (s - y)^2)^{3/2} ds, delta = lambda/2
    lam = W.LAMBDA_100GHZ
    L = m * lam / 4
    val, _ = integrate.quad(lambda s: x / (x * x + (s - y) ** 2) ** 1.5, -L, L,
                            points=[y] if -L < y < L else None, epsrel=1e-13, epsabs=0)
    assert cf.power_eq4(x, y, m, lam) == pytest.approx(val / (lam / 2), rel=1e-10)
    arr = W.ula(m, lam, W.AMP_PNUSW)
    assert cf.diag_ula(arr, x, y, m) == pytest.approx(val / (lam / 2), rel=1e-10)


def test_eq5_is_the_limit_of_eq4():
    lam = W.LAMBDA_100GHZ
    for x in (1.0, 3.0, 9.5):
        assert cf.power_eq4(x, 0.7, 1e12, lam) == pytest.approx(cf.power_limit_eq5(x, lam), rel=1e-9)


def test_eq8_is_the_limit_of_eq6():
    lam = W.LAMBDA_100GHZ
    for (xi, yi, xj, yj) in [(2.0, 0.5, 4.0, 1.7), (5.0, -1.0, 1.2, 3.0), (1.0, 0.0, 1.0001, 9.0)]:
        a = cf.rho_eq6(xi, yi, xj, yj, 1e13, lam)
        b = cf.rho_limit_eq8(xi, yi, xj, yj, lam)
        assert abs(a - b) < 1e-9 * abs(b) + 1e-15


def test_eq6_sgn_convention():
    # eq. (7): sgn(0) = -1; eq. (6) has magnitude ||x_i| - |x_j|| so equal-x users give 0
    assert cf.sgn(0.0) == -1.0 and cf.sgn(-2.0) == -1.0 and cf.sgn(1e-300) == 1.0
    assert cf.rho_eq6(2.0, 0.0, 2.0, 1.0, 4096, 0.003) == 0
    # swapping users conjugates rho (Hermitian)
    a = cf.rho_eq6(2.0, 0.5, 4.0, 1.7, 65536, 0.003)
    b = cf.rho_eq6(4.0, 1.7, 2.0, 0.5, 65536, 0.003)
    assert abs(a - np.conj(b)) < 1e-15


def test_general_spacing_matches_verbatim_at_half_lambda():
    lam = W.LAMBDA_100GHZ
    m = 65536
    arr = W.ula(m, lam, W.AMP_PNUSW)
    u = _users([(2.0, 0.5), (4.0, 1.7), (1.2, -0.8), (6.0, 3.0)])
    g = cf.gram_closedform(arr, u)
    for i in range(4):
        assert g[i, i].real == pytest.approx(cf.power_eq4(u[i, 0], u[i, 1], m, lam), rel=1e-13)
        for j in range(4):
            if i != j:
                want = cf.rho_eq6(u[i, 0], u[i, 1], u[j, 0], u[j, 1], m, lam) * math.sqrt(g[i, i].real * g[j, j].real)
                assert abs(g[i, j] - want) < 1e-12 * abs(want)
    assert np.allclose(g, g.conj().T, rtol=1e-13, atol=0)


@pytest.mark.parametrize("n", [256, 4096])
def test_freespace_diagonal_vs_quadrature_and_sum(n):
    lam = W.LAMBDA_28GHZ
    arr = W.ula(n, lam)
    L = n * arr.spacing / 2
    u = _users([(5.0, 0.3), (20.0, -12.0)])
    c = (lam / (4 * math.pi)) ** 2
    g = ch.gram_exact(arr, u)
    for i in range(2):
        x, y = u[i, 0], u[i, 1]
        val, _ = integrate.quad(lambda s: 1.0 / (x * x + (s - y) ** 2), -L, L, epsrel=1e-13, epsabs=0)
        assert cf.diag_ula(arr, x, y, n) == pytest.approx(c * val / arr.spacing, rel=1e-11)
        # midpoint rule vs the direct sum
        assert g[i, i].real == pytest.approx(cf.diag_ula(arr, x, y, n), rel=1e-6)


def test_freespace_offdiag_vs_exact():
    # Derived free-space stationary-phase term: agrees with the exact Gram when the
    # stationary point is deep inside the aperture, up to the endpoint terms of the
    # 1/r amplitude (a floor of a few 1e-4 normwise at this size).
    lam = W.LAMBDA_28GHZ
    n = 262144
    arr = W.ula(n, lam)
    u = _users([(5.0, 1.0), (12.0, 4.0), (8.0, -3.0)])
    g = ch.gram_exact(arr, u)
    gc = cf.gram_closedform(arr, u, variant=cf.VARIANT_GATED)
    assert ch.normwise_error(gc, g) < 1e-3
    for i, j in [(0, 1), (1, 2)]:
        assert abs(np.angle(g[i, j] / gc[i, j])) < 0.05


def test_gated_variant_zeroes_outside_aperture():
    lam = W.LAMBDA_28GHZ
    arr = W.ula(256, lam)   # 1.37 m aperture
    u = _users([(5.0, 1.0), (12.0, 4.0)])   # stationary point at y* = -1.14 m: outside
    gp = cf.gram_closedform(arr, u, variant=cf.VARIANT_PAPER)
    gg = cf.gram_closedform(arr, u, variant=cf.VARIANT_GATED)
    assert gg[0, 1] == 0 and gp[0, 1] != 0
    assert gg[0, 0] == gp[0, 0]


def test_upa_freespace_diagonal_vs_sum_and_dblquad():
    lam = W.LAMBDA_100GHZ_UPA
    arr = W.ArraySpec(W.GEOM_UPA, 128, 96, lam / 2, lam)
    u = np.array([[2.0, 0.05, -0.03], [4.0, -1.0, 0.5]])
    g = ch.gram_exact(arr, u)
    c = (lam / (4 * math.pi)) ** 2
    ly, lz = 128 * lam / 4, 96 * lam / 4
    for i in range(2):
        x, y, z = u[i]
        val, _ = integrate.dblquad(lambda v, s: 1.0 / (x * x + (s - y) ** 2 + (v - z) ** 2),
                                   -ly, ly, -lz, lz, epsabs=0, epsrel=1e-12)
        d = cf.diag_upa(arr, u[i])
        assert d == pytest.approx(c * val / arr.spacing ** 2, rel=1e-9)
        assert g[i, i].real == pytest.approx(d, rel=1e-5)


def test_upa_pnusw_diagonal_solid_angle():
    lam = W.LAMBDA_100GHZ_UPA
    arr = W.ArraySpec(W.GEOM_UPA, 64, 80, lam / 2, lam, W.AMP_PNUSW)
    u = np.array([[0.3, 0.02, -0.01], [1.0, -0.2, 0.3]])
    ly, lz = 64 * lam / 4, 80 * lam / 4
    g = ch.gram_exact(arr, u)
    for i in range(2):
        x, y, z = u[i]
        val, _ = integrate.dblquad(lambda v, s: x / (x * x + (s - y) ** 2 + (v - z) ** 2) ** 1.5,
                                   -ly, ly, -lz, lz, epsabs=0, epsrel=1e-12)
        assert cf.diag_upa(arr, u[i]) == pytest.approx(val / arr.spacing ** 2, rel=1e-9)
        assert g[i, i].real == pytest.approx(cf.diag_upa(arr, u[i]), rel=1e-4)


@pytest.mark.slow
def test_upa_offdiag_vs_exact_large_panel():
    # 2-D stationary phase: phase offset -pi/2, magnitude (lambda/4pi)^2 lambda / (delta^2 |dx|).
    lam = W.LAMBDA_100GHZ_UPA
    arr = W.ArraySpec(W.GEOM_UPA, 1536, 1536, lam / 2, lam)   # 2.3 m panel
    u = np.array([[0.6, 0.05, 0.02], [1.1, 0.12, -0.04]])
    g = ch.gram_exact(arr, u, chunk=1 << 18)
    gc = cf.gram_closedform(arr, u, variant=cf.VARIANT_GATED)
    assert gc[0, 1] != 0
    # |rho| = 1.5e-3 here; the edge terms of the finite panel leave ~8 % (phase 0.07 rad),
    # while a wrong pi/4 offset or a dropped 2 pi / lambda factor would be off by far more.
    assert abs(g[0, 1] - gc[0, 1]) < 0.15 * abs(gc[0, 1])
    assert abs(np.angle(g[0, 1] / gc[0, 1])) < 0.1
