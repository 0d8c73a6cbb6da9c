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

Pins (tests/test_oracle_closedform.py): eq. (4) against the direct sum and
against adaptive quadrature of the integrand; eq. (5) as the M -> inf limit;
eq. (6) against the exact Gram at large M; eq. (8) as the limit of eq. (6);
free-space and UPA diagonals against quadrature.
"""
from __future__ import annotations

import numpy as np
from scipy import integrate

from workloads import AMP_FREESPACE, AMP_PNUSW, GEOM_ULA, GEOM_UPA, ArraySpec

from .geometry import perpendicular_distance

VARIANT_PAPER = 0
VARIANT_GATED = 1


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
