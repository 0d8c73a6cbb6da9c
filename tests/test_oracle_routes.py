"""Pins of the route thresholds of the closed forms UNIFORM and GATED_QUAD
(ULA extensions beyond the paper's eqs. (6)/(23)) against the definition of a
Gram entry, the direct sum over the N elements (Sec. III).

Each threshold of the oracle's route choice is straddled by a pair of users
placed just on either side of it:
  * the slow-phase limit (QUAD_MAX_PANELS panels of QUAD_RAD_PER_PANEL rad:
    at most 960 rad of phase over the aperture),
  * the broad stationary zone (Fresnel width sqrt(2 pi / |phi''(y*)|) against
    L / BROAD_FRACTION),
  * the quadrature budget of a broad pair (QUAD_NODES nodes per panel, at most
    N / 8 nodes),
  * the direct-sum size DIRECT_MAX_N.
The test asserts that the route changes across the threshold, and that on both
sides the entry agrees with the exact Gram (normwise, |dG_ij| / sqrt(G_ii G_jj))
within the variant's tolerance: 1e-7 for a pair on a numeric route (quadrature
or direct sum), 5e-4 for a pair on UNIFORM's analytic route.  GATED_QUAD has no
accuracy claim on its analytic pairs (they are the paper's gated term); its
numeric pairs are held to the same 1e-7.  A change of a threshold is then
judged against the definition, not against the GPU kernel.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import channel as ch
from oracle import closedform as cf

LAM = W.LAMBDA_28GHZ
K_WAVE = 2.0 * math.pi / LAM
TOL_NUMERIC = 1e-7
TOL_UNIFORM_ANALYTIC = 5e-4


def _on_line(ys, th, a, b):
    """Two users on the line through the array point (0, ys) at angle th from broadside,
    at distances a and b from it: the stationary point of the pair is ys."""
    return (a * math.cos(th), ys + a * math.sin(th)), (b * math.cos(th), ys + b * math.sin(th))


def _broadness(ui, uj, n):
    """Fresnel width of the pair's stationary zone over L / BROAD_FRACTION (L the half-aperture):
    at least 1 for a broad zone."""
    (xi, yi), (xj, yj) = ui, uj
    ys = (yi * xj - xi * yj) / (xj - xi)
    a, b = math.hypot(xi, ys - yi), math.hypot(xj, ys - yj)
    p2 = K_WAVE * (xi * xi / a ** 3 - xj * xj / b ** 3)
    return math.sqrt(2.0 * math.pi / abs(p2)) / (n * (LAM / 2) / 2.0) * cf.BROAD_FRACTION


def _route(ui, uj, n):
    return cf.numeric_route(LAM / 2, LAM, ui[0], ui[1], uj[0], uj[1], n)


def _errors(ui, uj, n):
    """Normwise errors of the UNIFORM and GATED_QUAD entries against the exact Gram, and GATED's entry."""
    arr = W.ula(n, LAM)
    users = np.array([[ui[0], ui[1], 0.0], [uj[0], uj[1], 0.0]])
    g = ch.gram_exact(arr, users)
    s = math.sqrt(g[0, 0].real * g[1, 1].real)
    gu = cf.gram_closedform(arr, users, n, cf.VARIANT_UNIFORM)
    gq = cf.gram_closedform(arr, users, n, cf.VARIANT_GATED_QUAD)
    gg = cf.gram_closedform(arr, users, n, cf.VARIANT_GATED)
    return abs(gu[0, 1] - g[0, 1]) / s, abs(gq[0, 1] - g[0, 1]) / s, gq[0, 1], gg[0, 1]


def _check_side(ui, uj, n, numeric):
    route, _ = _route(ui, uj, n)
    assert (route != cf.ROUTE_NONE) == numeric, (route, numeric)
    e_uni, e_gq, v_gq, v_gated = _errors(ui, uj, n)
    if numeric:
        assert e_uni < TOL_NUMERIC and e_gq < TOL_NUMERIC, (e_uni, e_gq)
    else:
        assert e_uni < TOL_UNIFORM_ANALYTIC, e_uni
        assert v_gq == v_gated   # GATED_QUAD keeps the paper's gated term on analytic pairs
    return route


@pytest.mark.parametrize("n", [4096, 65536, 262144])
def test_slow_phase_threshold(n):
    # user j moves away from user i; the panel count k |u_i - u_j| span / 120 crosses 8
    ui = (10.0, 1.0)
    direction = (0.6, 0.8)

    def panels_exact(sep):
        uj = (ui[0] + sep * direction[0], ui[1] + sep * direction[1])
        xm, ym = 0.5 * (ui[0] + uj[0]), 0.5 * (ui[1] + uj[1])
        L = n * (LAM / 2) / 2.0
        span = math.atan((L - ym) / xm) - math.atan((-L - ym) / xm)
        return K_WAVE * sep * span / cf.QUAD_RAD_PER_PANEL

    lo, hi = 1e-4, 10.0
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        lo, hi = (mid, hi) if panels_exact(mid) < cf.QUAD_MAX_PANELS else (lo, mid)
    for fac, numeric in ((0.995, True), (1.005, False)):
        sep = lo * fac
        uj = (ui[0] + sep * direction[0], ui[1] + sep * direction[1])
        p = cf.quad_panels(LAM / 2, LAM, ui[0], ui[1], uj[0], uj[1], n)
        assert p == (cf.QUAD_MAX_PANELS if numeric else cf.QUAD_MAX_PANELS + 1)
        # the far side of this threshold must not be rescued by the broad-zone rule
        if not numeric:
            assert _broadness(ui, uj, n) < 1.0 or p * cf.QUAD_NODES * 8 > n
        _check_side(ui, uj, n, numeric)


@pytest.mark.parametrize("n,ys,th,a", [(262144, 500.0, math.radians(-85.0), 520.0),
                                       (65536, 100.0, math.radians(-85.0), 400.0)])
def test_broad_zone_threshold(n, ys, th, a):
    # users on one line through the array point ys: the Fresnel width of their stationary
    # zone grows as 1/a - 1/b shrinks; bisect b to the width L / BROAD_FRACTION
    def excess(b):
        ui, uj = _on_line(ys, th, a, b)
        return _broadness(ui, uj, n) - 1.0

    lo, hi = a * (1 + 1e-9), 3.0 * a
    assert excess(lo) > 0 > excess(hi)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if excess(mid) > 0 else (lo, mid)
    b0 = lo
    for fac, numeric in ((0.98, True), (1.02, False)):
        b = 1.0 / (1.0 / a - fac * (1.0 / a - 1.0 / b0))   # scales 1/a - 1/b by fac
        ui, uj = _on_line(ys, th, a, b)
        p = cf.quad_panels(LAM / 2, LAM, ui[0], ui[1], uj[0], uj[1], n)
        # neither slow-phase nor over the budget: only the width decides
        assert cf.QUAD_MAX_PANELS < p and p * cf.QUAD_NODES * 8 <= n, p
        assert abs(ys) < n * (LAM / 2) / 2.0   # stationary point on the aperture
        _check_side(ui, uj, n, numeric)


def test_quadrature_budget_threshold():
    # a broad pair (stationary point inside the aperture) whose quadrature needs about N / 8
    # nodes near N = 27000: the panel count grows with the aperture's angular span, so the
    # budget flips between two neighbouring N while the zone stays broad
    ui, uj = _on_line(-25.283, 1.4958, 95.4606, 103.43317)
    ok = lambda n: cf.quad_panels(LAM / 2, LAM, ui[0], ui[1], uj[0], uj[1], n) * cf.QUAD_NODES * 8 <= n
    lo, hi = 26495, 27149
    assert ok(lo) != ok(hi)
    while hi - lo > 1:
        mid = (lo + hi) // 2
        lo, hi = (mid, hi) if ok(mid) == ok(lo) else (lo, mid)
    for n in (lo, hi):
        assert _broadness(ui, uj, n) > 1.0   # broad on both sides
        p = cf.quad_panels(LAM / 2, LAM, ui[0], ui[1], uj[0], uj[1], n)
        assert p > cf.QUAD_MAX_PANELS
        _check_side(ui, uj, n, ok(n))


def test_direct_sum_size_threshold():
    # a slow-phase pair: the direct sum up to DIRECT_MAX_N elements, the quadrature above
    ui, uj = (8.0, -2.0), (8.02, -1.97)
    n0 = cf.DIRECT_MAX_N
    r0, p0 = _route(ui, uj, n0)
    r1, p1 = _route(ui, uj, n0 + 1)
    assert r0 == cf.ROUTE_DIRECT and r1 == cf.ROUTE_QUAD
    assert p1 * cf.QUAD_NODES < n0 + 1   # the quadrature is the cheaper route above the limit
    for n in (n0, n0 + 1):
        e_uni, e_gq, _, _ = _errors(ui, uj, n)
        assert e_uni < TOL_NUMERIC and e_gq < TOL_NUMERIC, (n, e_uni, e_gq)


def test_direct_route_is_the_definition():
    # on the direct route the entry is the exact sum itself (same terms, one pair at a time)
    ui, uj = (12.0, 3.0), (12.3, 3.4)
    n = 1024
    assert _route(ui, uj, n)[0] == cf.ROUTE_DIRECT
    e_uni, e_gq, _, _ = _errors(ui, uj, n)
    assert e_uni < 1e-13 and e_gq < 1e-13
