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


# ---------------------------------------------------------------- variant UNIFORM

def test_fresnel_wrapper_is_the_quadratic_phase_integral():
    # F(s) = int_0^s e^{j sigma t^2/2} dt: direct quadrature, the infinite limit, oddness
    for sigma in (1.0, -1.0):
        for s in (0.3, 2.5, 7.0):
            re, _ = integrate.quad(lambda t: math.cos(sigma * t * t / 2), 0, s, epsabs=0, epsrel=1e-13, limit=200)
            im, _ = integrate.quad(lambda t: math.sin(sigma * t * t / 2), 0, s, epsabs=0, epsrel=1e-13, limit=200)
            assert abs(cf.fresnel_f(s, sigma) - (re + 1j * im)) < 1e-12
            assert cf.fresnel_f(-s, sigma) == pytest.approx(-cf.fresnel_f(s, sigma), abs=1e-15)
        lim = math.sqrt(math.pi / 2) * complex(math.cos(math.pi / 4), sigma * math.sin(math.pi / 4))
        assert abs(cf.fresnel_f(1e7, sigma) - lim) < 1e-7


@pytest.mark.parametrize("amp", [W.AMP_FREESPACE, W.AMP_PNUSW])
def test_aperture_integral_pins(amp):
    lam = W.LAMBDA_28GHZ
    n = 4096
    arr = W.ula(n, lam, amp)
    L = n * arr.spacing / 2
    # zero separation: the quadrature in the midpoint's angle equals the analytic diagonal
    for x, y in ((3.0, 0.5), (12.0, -4.0), (0.8, 11.0)):
        v = cf.aperture_integral(arr, x, y, x, y, n, 1)
        assert v.real == pytest.approx(cf.diag_ula(arr, x, y, n), rel=1e-12) and abs(v.imag) < 1e-14 * v.real
    # a slow pair: the same integral by adaptive quadrature in y
    xi, yi, xj, yj = 9.0, 2.0, 9.07, 2.05
    k = 2 * math.pi / lam

    def integrand(yv, part):
        a, b = math.hypot(xi, yv - yi), math.hypot(xj, yv - yj)
        f = (arr.beta0 * math.sqrt(xi * xj) / (a * b) ** 1.5) if amp == W.AMP_PNUSW else (lam / (4 * math.pi)) ** 2 / (a * b)
        return f * (math.cos(k * (a - b)) if part == 0 else math.sin(k * (a - b)))
    re, _ = integrate.quad(integrand, -L, L, args=(0,), points=[yi], epsabs=0, epsrel=1e-12, limit=400)
    im, _ = integrate.quad(integrand, -L, L, args=(1,), points=[yi], epsabs=0, epsrel=1e-12, limit=400)
    p = cf.slow_pair_panels(arr, xi, yi, xj, yj, n)
    assert p >= 1
    v = cf.aperture_integral(arr, xi, yi, xj, yj, n, p)
    assert abs(v - (re + 1j * im) / arr.spacing) < 1e-10 * abs(v)


def test_slow_pairs_match_the_exact_sum():
    # users a few centimetres to 0.3 m apart: no stationary-phase regime; the quadrature plus the
    # discrete end corrections reproduces the exact discrete sum
    lam = W.LAMBDA_28GHZ
    rng = np.random.default_rng(3)
    for n in (256, 4096, 65536):
        arr = W.ula(n, lam)
        for sep in (0.0, 0.02, 0.15, 0.3):
            ang = rng.uniform(0, 2 * np.pi)
            u = _users([(7.0, -2.0), (7.0 + sep * math.cos(ang), -2.0 + sep * math.sin(ang))])
            g = ch.gram_exact(arr, u)
            assert cf.slow_pair_panels(arr, u[0, 0], u[0, 1], u[1, 0], u[1, 1], n) > 0
            gu = cf.gram_closedform(arr, u, n, cf.VARIANT_UNIFORM)
            assert ch.normwise_error(gu, g) < 1e-6, (n, sep)
            gg = cf.gram_closedform(arr, u, n, cf.VARIANT_GATED)
            if sep > 0:
                assert ch.normwise_error(gg, g) > 1e-3   # the paper's form has no answer here


@pytest.mark.parametrize("n", [256, 4096])
def test_uniform_matches_exact_on_sweep_drops(n):
    arr0, drops, _ = W.sweep(400)
    arr = arr0.with_n(n)
    errs_u, errs_g = [], []
    for d in range(0, 400, 20):
        u = drops.users_of(d)
        g = ch.gram_exact(arr, u)
        errs_u.append(ch.normwise_error(cf.gram_closedform(arr, u, n, cf.VARIANT_UNIFORM), g))
        errs_g.append(ch.normwise_error(cf.gram_closedform(arr, u, n, cf.VARIANT_GATED), g))
    assert max(errs_u) < 1e-4
    assert np.median(errs_u) < 1e-3 * np.median(errs_g)


def test_uniform_is_continuous_as_the_stationary_point_crosses_the_end():
    # move user j so that y* sweeps through the top end: the gated form jumps by the whole
    # stationary-phase term, the uniform form follows the exact sum
    lam = W.LAMBDA_28GHZ
    n = 4096
    arr = W.ula(n, lam)
    L = n * arr.spacing / 2
    xi, yi, xj = 6.0, 2.0, 18.0
    worst_u, worst_g = 0.0, 0.0
    for ys in list(np.linspace(L - 0.6, L + 0.6, 13)) + [L + 1e-6, L - 1e-9]:
        yj = ys + (yi - ys) * xj / xi   # user j on the line through user i and (0, ys)
        u = _users([(xi, yi), (xj, yj)])
        g = ch.gram_exact(arr, u)
        worst_u = max(worst_u, ch.normwise_error(cf.gram_closedform(arr, u, n, cf.VARIANT_UNIFORM), g))
        worst_g = max(worst_g, ch.normwise_error(cf.gram_closedform(arr, u, n, cf.VARIANT_GATED), g))
    assert worst_u < 1e-5 and worst_g > 3e-3


def test_uniform_far_outside_is_the_discrete_end_series():
    # stationary point far off the aperture: what remains are the two end contributions, i.e. the
    # geometric series of a locally linear phase at each end
    lam = W.LAMBDA_28GHZ
    n = 1024
    arr = W.ula(n, lam)
    d = arr.spacing
    k = 2 * math.pi / lam
    y_top = (n - 1) * d / 2
    xi, yi, xj, yj = 44.6, -0.1, 14.0, -19.1
    u = _users([(xi, yi), (xj, yj)])

    def geo(ye, side):
        a, b = math.hypot(xi, ye - yi), math.hypot(xj, ye - yj)
        th = side * k * ((ye - yi) / a - (ye - yj) / b) * d
        return (lam / (4 * math.pi)) ** 2 / (a * b) * np.exp(1j * k * (a - b)) / (1 - np.exp(-1j * th))
    s_geo = geo(y_top, 1.0) + geo(-y_top, -1.0)
    gu = cf.gram_closedform(arr, u, n, cf.VARIANT_UNIFORM)[0, 1]
    g = ch.gram_exact(arr, u)[0, 1]
    assert abs(gu - s_geo) < 2e-4 * abs(s_geo)
    assert abs(gu - g) < 2e-4 * abs(g)


def test_numeric_routes():
    lam = W.LAMBDA_28GHZ
    # the direct route is the definition of the entry for one pair
    arr = W.ula(60, lam)
    u = _users([(6.0, 1.0), (6.02, 1.01)])
    route, p = cf.numeric_route(arr.spacing, lam, 6.0, 1.0, 6.02, 1.01, 60)
    assert route == cf.ROUTE_DIRECT
    assert abs(cf.direct_sum(arr, 6.0, 1.0, 6.02, 1.01, 60) - ch.gram_exact(arr, u)[0, 1]) < 1e-12 * ch.gram_exact(arr, u)[0, 0].real
    # a broad stationary zone (nearly equal perpendicular distances, a 1.4 km aperture): the uniform
    # expansion misses the non-quadratic phase, the quadrature route reproduces the exact sum
    n = 262144
    arr = W.ula(n, lam)
    xi, yi, xj, yj = 7.1, 3.0, 7.12, 0.5
    route, p = cf.numeric_route(arr.spacing, lam, xi, yi, xj, yj, n)
    assert route == cf.ROUTE_QUAD and p > cf.QUAD_MAX_PANELS
    g = ch.gram_exact(arr, _users([(xi, yi), (xj, yj)]))
    den = math.sqrt(g[0, 0].real * g[1, 1].real)
    v = cf.numeric_entry(arr, xi, yi, xj, yj, n, route, p)
    assert abs(v - g[0, 1]) < 1e-10 * den
    assert abs(cf.uniform_pair(arr, xi, yi, xj, yj, n) - g[0, 1]) > 1e-4 * den
    # a typical pair keeps the analytic route
    assert cf.numeric_route(arr.spacing, lam, 9.0, 4.0, 31.0, -12.0, n)[0] == cf.ROUTE_NONE


def test_uniform_matches_exact_at_the_largest_aperture():
    # the analytic route's residual grows with the aperture (stationary zones a few tenths of L wide,
    # below the numeric route's threshold, keep a few 1e-4 normwise at N = 262144)
    arr0, drops, _ = W.sweep(200)
    n = 262144
    arr = arr0.with_n(n)
    errs = [ch.normwise_error(cf.gram_closedform(arr, drops.users_of(d), n, cf.VARIANT_UNIFORM),
                              ch.gram_exact(arr, drops.users_of(d))) for d in range(0, 200, 25)]
    assert max(errs) < 1e-3 and np.median(errs) < 1e-4
