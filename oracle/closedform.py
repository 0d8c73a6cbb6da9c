"""Closed-form (stationary-phase) Gram used by the paper's modified ZF.

Paper formulas (PNUSW channel, ULA, spacing lambda/2, M antennas):
  eq. (4)  P_i / P ~= 2 beta0 / (lambda x_i) * S_i,
           S_i = (M lambda - 4 y_i) / sqrt(16 x_i^2 + (M lambda - 4 y_i)^2)
               + (M lambda + 4 y_i) / sqrt(16 x_i^2 + (M lambda + 4 y_i)^2)
  eq. (5)  P_i^lim / P = 4 beta0 / (lambda x_i)
  eq. (6)  rho_ij ~= sqrt(lambda) | |x_i| - |x_j| | / d_ij^{3/2} * S_i^{-1/2} S_j^{-1/2}
                     * exp(j sgn(|x_i| - |x_j|) (2 pi d_ij / lambda - pi / 4))
  eq. (7)  sgn(x) = -1 for x <= 0, +1 for x > 0
  eq. (8)  lim_{M->inf} rho_ij = sqrt(lambda) |cos gamma_ij| / (2 sqrt(d_ij)) * (same phase)
  eqs. (22)-(23)  G~_ii = P_i / P,  G~_ij = rho_ij sqrt(P_i P_j) / P      ("modified ZF")

Readings taken where the paper is silent:
  * General spacing delta: eq. (4) is the midpoint rule over the aperture
    [-L, L], L = M delta / 2, so G~_ii = beta0 / (delta x_i) * S_i with
    S_i = (L - y_i)/sqrt(x_i^2 + (L - y_i)^2) + (L + y_i)/sqrt(x_i^2 + (L + y_i)^2);
    at delta = lambda/2 this is eq. (4) exactly.  rho of eq. (6) has no delta.
  * cos gamma_ij in eq. (8) is (|x_i| - |x_j|) / d_ij (the angle between the
    user-user line and the array normal).
  * Free-space channel lambda/(4 pi r) (the benchmark workloads' model): the
    same midpoint integral gives G~_ii = (lambda/4pi)^2 / (delta x_i)
    [atan((L - y_i)/x_i) + atan((L + y_i)/x_i)] and the same stationary-phase
    step gives G~_ij = (lambda/4pi)^2 sqrt(lambda) / (delta sqrt(x_i x_j d_ij))
    * exp(j sgn(x_i - x_j)(2 pi d_ij/lambda - pi/4)).
  * UPA (paper: future work): the diagonal is the 2-D integral
    (1/delta^2) int int |h|^2 over the panel; the off-diagonal is the 2-D
    stationary-phase term, phase offset -pi/2 instead of -pi/4:
    free space  (lambda/4pi)^2 lambda / (delta^2 | |x_i| - |x_j| |),
    PNUSW       beta0 lambda / (delta^2 d_ij).
  * The stationary point is where the line through both users meets the
    array (ULA: y* = (x_j y_i - x_i y_j)/(x_j - x_i)).  Variant PAPER uses the
    formulas as printed, everywhere; variant GATED sets an off-diagonal to
    zero when that point lies outside the aperture.
  * |x_i| == |x_j| or coincident users: the off-diagonal is defined as 0.

Variant UNIFORM (ULA; an extension beyond the paper's formulas, not one of them):
  The paper's eq. (6) is the leading stationary-phase term of the aperture
  integral and stands alone; here the discrete sum
  S = sum_n f(y_n) e^{j phi(y_n)},  f = |h_i| |h_j|,  phi = k (r_i - r_j),
  is approximated uniformly in the position of the stationary point y*:
  * the continuum integral over the element cells [-L, L], L = N d / 2, by the
    uniform asymptotic expansion about y* (the exact change of variable
    phi(y) - phi* = sigma s^2 / 2, sigma = sgn phi''(y*), s of the sign of y - y*):
      I = G0 e^{j phi*} [F(s_b) - F(s_a)]
          + sum over the ends e = b (+), a (-) of
            +- e^{j phi(e)} [ f(e) / (j phi'(e)) - G0 / (j sigma s_e) ]
    with G0 = f(y*) / sqrt|phi''(y*)|, s_e = sgn(e - y*) sqrt(2 |phi(e) - phi*|)
    and F(s) = int_0^s e^{j sigma t^2 / 2} dt (Fresnel integrals).  With y* deep
    inside the aperture this is eq. (6)'s term plus the two end terms; with y*
    outside, the end terms alone; and it stays finite as y* crosses an end.
    x_i = x_j (no stationary point): the end terms alone.
  * S = I / d plus, at each end element y_e, the difference between the discrete
    half-infinite sum and its cell integral for a locally linear phase
    theta = phi'(y_e) d:  +- f(y_e) e^{j phi(y_e)} e^{+- j theta/2} / j
    [1 / (2 sin(theta/2)) - 1 / theta]  (+ at the top end y_top = (N-1) d / 2).
  * Numeric pairs (numeric_route): slow-phase pairs, for which k |u_i - u_j|
    times the angular span of the aperture seen from the pair's midpoint is at
    most QUAD_RAD_PER_PANEL * QUAD_MAX_PANELS radians (users a fraction of a
    metre apart: no asymptotic regime), and pairs whose stationary zone is broad
    (Fresnel width >= L / BROAD_FRACTION: the phase is far from quadratic over it)
    when that is affordable.  Their entry is the aperture integral
    (1/d) int_{-L}^{L} conj(h_i(y)) h_j(y) dy (the continuum limit of the sum,
    as eq. (4) is for the diagonal), evaluated by composite Gauss-Legendre
    quadrature in the angle theta seen from the midpoint (y = y_m + x_m tan theta),
    in panels over which the phase changes by at most QUAD_RAD_PER_PANEL rad,
    plus the same discrete end corrections; or the direct sum over the N
    elements (the definition itself) when the array has at most DIRECT_MAX_N
    elements or the sum costs no more than the quadrature.
  The diagonal is the closed form above.
"""
from __future__ import annotations

import numpy as np
from scipy import integrate, special

from workloads import AMP_FREESPACE, AMP_PNUSW, GEOM_ULA, GEOM_UPA, ArraySpec

from .geometry import perpendicular_distance

VARIANT_PAPER = 0
VARIANT_GATED = 1
VARIANT_UNIFORM = 2
VARIANT_GATED_QUAD = 3     # GATED, slow-phase pairs by the aperture quadrature (the learned correction's base)

QUAD_NODES = 64            # Gauss-Legendre nodes per panel
QUAD_RAD_PER_PANEL = 120.0  # phase change allowed over one panel (64 nodes resolve up to ~180 rad)
QUAD_MAX_PANELS = 8          # slow-phase pairs: at most 960 rad over the aperture
S_GUARD = 1e-2             # |s| below which the uniform end bracket is interpolated
BROAD_FRACTION = 2.0       # a stationary zone of Fresnel width >= L / BROAD_FRACTION is "broad"
DIRECT_MAX_N = 1024        # numeric pairs of arrays up to this size take the direct sum
ROUTE_NONE, ROUTE_DIRECT, ROUTE_QUAD = 0, 1, 2


def sgn(x):
    """eq. (7): -1 for x <= 0, +1 for x > 0."""
    return np.where(np.asarray(x) > 0, 1.0, -1.0)


# ---------------------------------------------------------------- paper, verbatim

def s_factor_eq4(x, y, m, lam):
    """Bracketed term of eq. (4) (M antennas, spacing lambda/2)."""
    a = m * lam - 4.0 * y
    b = m * lam + 4.0 * y
    return a / np.sqrt(16.0 * x * x + a * a) + b / np.sqrt(16.0 * x * x + b * b)


def power_eq4(x, y, m, lam, beta0=1.0):
    """eq. (4): P_i / P for the PNUSW ULA with lambda/2 spacing."""
    return 2.0 * beta0 / (lam * x) * s_factor_eq4(x, y, m, lam)


def power_limit_eq5(x, lam, beta0=1.0):
    """eq. (5): P_i^lim / P = 4 beta0 / (lambda x_i)."""
    return 4.0 * beta0 / (lam * x)


def rho_eq6(xi, yi, xj, yj, m, lam):
    """eq. (6): SPM correlation for the PNUSW ULA, with sgn of eq. (7)."""
    dx = np.abs(xi) - np.abs(xj)
    d = np.sqrt(dx * dx + (yi - yj) ** 2)
    mag = np.sqrt(lam) * np.abs(dx) / d ** 1.5 \
        / np.sqrt(s_factor_eq4(xi, yi, m, lam)) / np.sqrt(s_factor_eq4(xj, yj, m, lam))
    return mag * np.exp(1j * sgn(dx) * (2.0 * np.pi * d / lam - np.pi / 4.0))


def rho_limit_eq8(xi, yi, xj, yj, lam):
    """eq. (8): M -> inf limit of eq. (6); cos(gamma_ij) = (|x_i| - |x_j|) / d_ij."""
    dx = np.abs(xi) - np.abs(xj)
    d = np.sqrt(dx * dx + (yi - yj) ** 2)
    cos_g = dx / d
    return np.sqrt(lam) * np.abs(cos_g) / (2.0 * np.sqrt(d)) \
        * np.exp(1j * sgn(dx) * (2.0 * np.pi * d / lam - np.pi / 4.0))


# ---------------------------------------------------------------- general spacing

def s_factor(x, y, half_aperture):
    """S of eq. (4) written with the half-aperture L = M delta / 2."""
    L = half_aperture
    return (L - y) / np.sqrt(x * x + (L - y) ** 2) + (L + y) / np.sqrt(x * x + (L + y) ** 2)


def diag_ula(arr: ArraySpec, x, y, n):
    """G~_ii for a ULA of n elements: eq. (4)/P (PNUSW) or its free-space analogue."""
    L = n * arr.spacing / 2.0
    if arr.amp_model == AMP_PNUSW:
        return arr.beta0 / (arr.spacing * x) * s_factor(x, y, L)
    c = (arr.wavelength / (4.0 * np.pi)) ** 2
    return c / (arr.spacing * x) * (np.arctan((L - y) / x) + np.arctan((L + y) / x))


def _rect_integral_inv_r2(x, u1, u2, v1, v2):
    """int_{u1}^{u2} int_{v1}^{v2} du dv / (x^2 + u^2 + v^2), inner integral in closed form."""
    def inner(u):
        a = np.sqrt(x * x + u * u)
        return (np.arctan(v2 / a) - np.arctan(v1 / a)) / a
    pts = [p for p in (0.0,) if u1 < p < u2]
    val, _ = integrate.quad(inner, u1, u2, points=pts or None, epsabs=0.0, epsrel=1e-13, limit=200)
    return val


def _solid_angle_rect(x, u1, u2, v1, v2):
    """Solid angle of the rectangle [u1,u2]x[v1,v2] seen from height x above its plane."""
    def f(u, v):
        return np.arctan(u * v / (x * np.sqrt(x * x + u * u + v * v)))
    return f(u2, v2) - f(u1, v2) - f(u2, v1) + f(u1, v1)


def diag_upa(arr: ArraySpec, user):
    """G~_ii for the UPA: (1/delta^2) times the panel integral of |h|^2."""
    x, y, z = float(abs(user[0])), float(user[1]), float(user[2])
    ly = arr.n_y * arr.spacing / 2.0
    lz = arr.n_z * arr.spacing / 2.0
    if arr.amp_model == AMP_PNUSW:
        return arr.beta0 / arr.spacing ** 2 * _solid_angle_rect(x, -ly - y, ly - y, -lz - z, lz - z)
    c = (arr.wavelength / (4.0 * np.pi)) ** 2
    return c / arr.spacing ** 2 * _rect_integral_inv_r2(x, -ly - y, ly - y, -lz - z, lz - z)


def stationary_point(ui, uj):
    """Where the line through two users (perpendicular distances xi, xj) meets the array."""
    xi, xj = ui[0], uj[0]
    return [(ui[c] * xj - uj[c] * xi) / (xj - xi) for c in range(1, len(ui))]


def _amp_product(arr: ArraySpec, xp_i, xp_j, ri, rj):
    """|h_i| |h_j| at distances ri, rj (free space or PNUSW, eq. (3))."""
    if arr.amp_model == AMP_PNUSW:
        return arr.beta0 * np.sqrt(xp_i * xp_j) / (ri * rj) ** 1.5
    return (arr.wavelength / (4.0 * np.pi)) ** 2 / (ri * rj)


def quad_panels(spacing, lam, xp_i, y_i, xp_j, y_j, n):
    """Panels of QUAD_NODES nodes for the aperture quadrature: |d phi / d theta| <= k |u_i - u_j|."""
    k = 2.0 * np.pi / lam
    L = n * spacing / 2.0
    xm, ym = 0.5 * (xp_i + xp_j), 0.5 * (y_i + y_j)
    span = np.arctan((L - ym) / xm) - np.arctan((-L - ym) / xm)
    v = k * np.hypot(xp_i - xp_j, y_i - y_j) * span
    return max(1, int(np.ceil(v / QUAD_RAD_PER_PANEL)))


def numeric_route(spacing, lam, xp_i, y_i, xp_j, y_j, n):
    """(route, panels): route ROUTE_DIRECT / ROUTE_QUAD for a pair the closed forms UNIFORM and GATED_QUAD
    evaluate numerically, ROUTE_NONE otherwise.  Numeric pairs: slow-phase pairs (<= QUAD_MAX_PANELS
    panels) and pairs whose stationary zone is broad (Fresnel width sqrt(2 pi / |phi''(y*)|) >=
    L / BROAD_FRACTION, or x_i == x_j) when the quadrature costs at most N / 8 nodes; the direct sum over
    the N elements is used when N <= DIRECT_MAX_N or it costs no more than the quadrature."""
    p = quad_panels(spacing, lam, xp_i, y_i, xp_j, y_j, n)
    L = n * spacing / 2.0
    broad = True
    if xp_i != xp_j:
        k = 2.0 * np.pi / lam
        ys = (y_i * xp_j - xp_i * y_j) / (xp_j - xp_i)
        a, b = np.hypot(xp_i, ys - y_i), np.hypot(xp_j, ys - y_j)
        p2 = k * (xp_i ** 2 / a ** 3 - xp_j ** 2 / b ** 3)
        broad = p2 == 0.0 or 2.0 * np.pi / abs(p2) >= (L / BROAD_FRACTION) ** 2
    if p <= QUAD_MAX_PANELS or (broad and p * QUAD_NODES * 8 <= n):
        return (ROUTE_DIRECT if n <= max(p * QUAD_NODES, DIRECT_MAX_N) else ROUTE_QUAD), p
    return ROUTE_NONE, 0


def slow_pair_panels(arr: ArraySpec, xp_i, y_i, xp_j, y_j, n):
    """Panels of the aperture quadrature for a slow-phase pair, 0 for a fast-phase pair."""
    p = quad_panels(arr.spacing, arr.wavelength, xp_i, y_i, xp_j, y_j, n)
    return p if p <= QUAD_MAX_PANELS else 0


def direct_sum(arr: ArraySpec, xp_i, y_i, xp_j, y_j, n):
    """sum_n conj(h_i(y_n)) h_j(y_n) over the elements (the definition, for one pair)."""
    k = 2.0 * np.pi / arr.wavelength
    y = (np.arange(n) - (n - 1) / 2.0) * arr.spacing
    ri, rj = np.hypot(xp_i, y - y_i), np.hypot(xp_j, y - y_j)
    return np.sum(_amp_product(arr, xp_i, xp_j, ri, rj) * np.exp(1j * k * (ri - rj)))


def numeric_entry(arr: ArraySpec, xp_i, y_i, xp_j, y_j, n, route, panels):
    if route == ROUTE_DIRECT:
        return direct_sum(arr, xp_i, y_i, xp_j, y_j, n)
    return aperture_integral(arr, xp_i, y_i, xp_j, y_j, n, panels) \
        + discrete_end_corrections(arr, xp_i, y_i, xp_j, y_j, n)


def aperture_integral(arr: ArraySpec, xp_i, y_i, xp_j, y_j, n, panels):
    """(1/d) int_{-L}^{L} conj(h_i(y)) h_j(y) dy by composite Gauss-Legendre in the midpoint's angle."""
    k = 2.0 * np.pi / arr.wavelength
    L = n * arr.spacing / 2.0
    xm, ym = 0.5 * (xp_i + xp_j), 0.5 * (y_i + y_j)
    ta, tb = np.arctan((-L - ym) / xm), np.arctan((L - ym) / xm)
    nodes, weights = np.polynomial.legendre.leggauss(QUAD_NODES)
    edges = ta + (tb - ta) * np.arange(panels + 1) / panels
    total = 0.0 + 0.0j
    for a, b in zip(edges[:-1], edges[1:]):
        th = 0.5 * (a + b) + 0.5 * (b - a) * nodes
        y = ym + xm * np.tan(th)
        jac = xm / np.cos(th) ** 2
        ri, rj = np.hypot(xp_i, y - y_i), np.hypot(xp_j, y - y_j)
        total += 0.5 * (b - a) * np.sum(weights * jac * _amp_product(arr, xp_i, xp_j, ri, rj) * np.exp(1j * k * (ri - rj)))
    return total / arr.spacing


def fresnel_f(s, sigma):
    """F(s) = int_0^s e^{j sigma t^2 / 2} dt from the Fresnel integrals C and S (scipy)."""
    sv, cv = special.fresnel(s / np.sqrt(np.pi))
    return np.sqrt(np.pi) * (cv + 1j * sigma * sv)


def uniform_pair(arr: ArraySpec, xp_i, y_i, xp_j, y_j, n):
    """Entry (i, j) of variant UNIFORM for a fast-phase pair (see the module notes)."""
    k = 2.0 * np.pi / arr.wavelength
    d = arr.spacing
    L = n * d / 2.0
    y_top = (n - 1) * d / 2.0

    def dist(y):
        return np.hypot(xp_i, y - y_i), np.hypot(xp_j, y - y_j)

    def phi(y):
        a, b = dist(y)
        return k * (a - b)

    def dphi(y):
        a, b = dist(y)
        return k * ((y - y_i) / a - (y - y_j) / b)

    def f(y):
        a, b = dist(y)
        return _amp_product(arr, xp_i, xp_j, a, b)

    ends = ((L, 1.0), (-L, -1.0))
    integral = 0.0 + 0.0j
    if xp_i == xp_j:
        for e, se in ends:
            integral += se * f(e) * np.exp(1j * phi(e)) / (1j * dphi(e))
    else:
        ys = (y_i * xp_j - xp_i * y_j) / (xp_j - xp_i)
        a, b = dist(ys)
        p2 = k * (xp_i ** 2 / a ** 3 - xp_j ** 2 / b ** 3)
        sigma = 1.0 if p2 > 0 else -1.0
        g0 = f(ys) / np.sqrt(abs(p2))
        ph = phi(ys)

        ai_s, aj_s = dist(ys)

        def s_of(y):
            # phi(y) - phi* from r(y) - r(y*) = (y - y*)(y + y* - 2 y_u) / (r(y) + r(y*)), which keeps its
            # relative precision as y -> y* (the plain difference of the phases would not)
            ai, aj = dist(y)
            dr = (y - ys) * ((y + ys - 2.0 * y_i) / (ai + ai_s) - (y + ys - 2.0 * y_j) / (aj + aj_s))
            return np.copysign(np.sqrt(2.0 * k * abs(dr)), y - ys)

        def bracket(y):
            # the end term minus its stationary-point singularity (both diverge as y -> y*; the difference is smooth)
            return np.exp(1j * phi(y)) * (f(y) / (1j * dphi(y)) - g0 / (1j * sigma * s_of(y)))

        for e, se in ends:
            s_e = s_of(e)
            if abs(s_e) < S_GUARD:
                # too close to the stationary point for the difference: interpolate it linearly in y
                h = S_GUARD / np.sqrt(abs(p2))
                bm, bp = bracket(ys - h), bracket(ys + h)
                br = bm + (e - (ys - h)) / (2.0 * h) * (bp - bm)
            else:
                br = bracket(e)
            integral += se * (g0 * np.exp(1j * ph) * fresnel_f(s_e, sigma) + br)
    return integral / d + discrete_end_corrections(arr, xp_i, y_i, xp_j, y_j, n)


def _half_cosec_minus_inverse(th):
    """1 / (2 sin(th/2)) - 1/th, by its series th/24 + 7 th^3/5760 + 31 th^5/967680 near 0."""
    if abs(th) < 1e-2:
        t2 = th * th
        return th * (1.0 / 24.0 + t2 * (7.0 / 5760.0 + t2 * 31.0 / 967680.0))
    return 1.0 / (2.0 * np.sin(th / 2.0)) - 1.0 / th


def discrete_end_corrections(arr: ArraySpec, xp_i, y_i, xp_j, y_j, n):
    """Sum minus cell integral at both end elements for a locally linear phase theta = phi'(y_e) d."""
    k = 2.0 * np.pi / arr.wavelength
    d = arr.spacing
    y_top = (n - 1) * d / 2.0
    total = 0.0 + 0.0j
    for e, side in ((y_top, 1.0), (-y_top, -1.0)):
        a, b = np.hypot(xp_i, e - y_i), np.hypot(xp_j, e - y_j)
        th = k * ((e - y_i) / a - (e - y_j) / b) * d
        total += side * _amp_product(arr, xp_i, xp_j, a, b) * np.exp(1j * k * (a - b)) \
            * np.exp(1j * side * th / 2.0) / 1j * _half_cosec_minus_inverse(th)
    return total


def gram_closedform(arr: ArraySpec, users: np.ndarray, n: int = None, variant: int = VARIANT_PAPER) -> np.ndarray:
    """Modified-ZF Gram G~ (eqs. (22)-(23)) for one drop; K x K complex128."""
    users = np.asarray(users, np.float64)
    k = users.shape[0]
    lam = arr.wavelength
    kw = 2.0 * np.pi / lam
    xp = perpendicular_distance(arr, users)
    g = np.zeros((k, k), np.complex128)
    if arr.geometry == GEOM_ULA:
        n = arr.n_y if n is None else int(n)
        L = n * arr.spacing / 2.0
        two_d = np.stack([xp, users[:, 1]], axis=-1)
        for i in range(k):
            g[i, i] = diag_ula(arr, xp[i], users[i, 1], n)
    else:
        assert arr.geometry == GEOM_UPA
        ly, lz = arr.n_y * arr.spacing / 2.0, arr.n_z * arr.spacing / 2.0
        two_d = np.stack([xp, users[:, 1], users[:, 2]], axis=-1)
        for i in range(k):
            g[i, i] = diag_upa(arr, users[i])
    if variant in (VARIANT_UNIFORM, VARIANT_GATED_QUAD):
        assert arr.geometry == GEOM_ULA, "variants UNIFORM and GATED_QUAD are defined for a ULA"
        g_sp = gram_closedform(arr, users, n, VARIANT_GATED) if variant == VARIANT_GATED_QUAD else None
        for i in range(k):
            for j in range(i + 1, k):
                route, p = numeric_route(arr.spacing, lam, xp[i], users[i, 1], xp[j], users[j, 1], n)
                if route != ROUTE_NONE:
                    v = numeric_entry(arr, xp[i], users[i, 1], xp[j], users[j, 1], n, route, p)
                elif variant == VARIANT_UNIFORM:
                    v = uniform_pair(arr, xp[i], users[i, 1], xp[j], users[j, 1], n)
                else:
                    v = g_sp[i, j]
                g[i, j] = v
                g[j, i] = np.conj(v)
        return g
    for i in range(k):
        for j in range(k):
            if i == j:
                continue
            dx = xp[i] - xp[j]
            d = float(np.linalg.norm(two_d[i] - two_d[j]))
            if dx == 0.0 or d == 0.0:
                continue
            if variant == VARIANT_GATED:
                sp = stationary_point(two_d[i], two_d[j])
                if arr.geometry == GEOM_ULA:
                    inside = abs(sp[0]) <= L
                else:
                    inside = abs(sp[0]) <= ly and abs(sp[1]) <= lz
                if not inside:
                    continue
            s = 1.0 if dx > 0 else -1.0
            if arr.geometry == GEOM_ULA:
                if arr.amp_model == AMP_PNUSW:
                    # eq. (6) with general-spacing S, then eq. (23)
                    rho = np.sqrt(lam) * abs(dx) / d ** 1.5 \
                        / np.sqrt(s_factor(xp[i], users[i, 1], L) * s_factor(xp[j], users[j, 1], L)) \
                        * np.exp(1j * s * (kw * d - np.pi / 4.0))
                    g[i, j] = rho * np.sqrt(g[i, i].real * g[j, j].real)
                else:
                    c = (lam / (4.0 * np.pi)) ** 2
                    g[i, j] = c * np.sqrt(lam) / (arr.spacing * np.sqrt(xp[i] * xp[j] * d)) \
                        * np.exp(1j * s * (kw * d - np.pi / 4.0))
            else:
                if arr.amp_model == AMP_PNUSW:
                    mag = arr.beta0 * lam / (arr.spacing ** 2 * d)
                else:
                    mag = (lam / (4.0 * np.pi)) ** 2 * lam / (arr.spacing ** 2 * abs(dx))
                g[i, j] = mag * np.exp(1j * s * (kw * d - np.pi / 2.0))
    return g


def gram_closedform_batch(arr: ArraySpec, drops, variant=VARIANT_PAPER, idx=None) -> list:
    out = []
    for d in (range(drops.n_drops) if idx is None else idx):
        n = int(drops.n_elems[d]) if arr.geometry == GEOM_ULA else None
        out.append(gram_closedform(arr, drops.users_of(d), n, variant))
    return out
