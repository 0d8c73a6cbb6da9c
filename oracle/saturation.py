"""Power / capacity saturation point (paper Sec. IV, Appendices B and C).

  eq. (10)-(11)  P_i / P_i^lim >= t  <=>  S_i / 2 >= t   (S_i from eq. (4))
  eq. (12)       at y_i = 0:  M >= 4 x_i t / (lambda sqrt(1 - t^2))
  eq. (13)-(14)  y_up^i = tau x_i + y_i,  y_down^i = -tau x_i + y_i,  tau = t / sqrt(1 - t^2)
  eq. (15)-(16)  y_up = max_i y_up^i,  y_down = min_i y_down^i
  eq. (17)       E[y_up] for x ~ U[x_min, x_max], y ~ U[y_min, y_max], K users
  eq. (18)       E[y_down] = y_min + y_max - E[y_up]
  eq. (19)-(20)  K -> inf limits (corner points)
  Appendix B     trapezoidal pdf of z_i = tau x_i + y_i, CDF of the max of K
                 draws and the expectation integral.

Readings:
  * eq. (17) prints "(2N+1)" in its fourth term; re-deriving it from the
    Appendix B integral gives (2K+1), which is used here (the test pins it
    against the integral and against Monte Carlo).
  * Appendix B writes z_i = x_i t / (1 - t^2) + y_i; the main text's
    tau = t / sqrt(1 - t^2) is used.
  * Saturation antenna count of a centred ULA: M_sat = (E y_up - E y_down) / delta
    (the span between the two saturation coordinates, as the paper draws its
    vertical line from the difference of eqs. (17) and (18)).
  * Empirical saturation (the paper only overlays the line on its curves):
    the first N, log-interpolated, where C(N) / C(N_max) >= 1 - eps.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, special


def tau(t):
    return t / math.sqrt(1.0 - t * t)


def power_ratio_eq11(x, y, m, lam):
    """Left-hand side of eq. (11): P_i / P_i^lim from eqs. (4)-(5)."""
    a = m * lam - 4.0 * y
    b = m * lam + 4.0 * y
    return a / (2.0 * np.sqrt(16.0 * x * x + a * a)) + b / (2.0 * np.sqrt(16.0 * x * x + b * b))


def m_single_user_eq12(x, t, lam):
    return 4.0 * x * t / (lam * math.sqrt(1.0 - t * t))


def y_bounds_eq15_16(users_xperp, users_y, t):
    """(y_up, y_down) of one drop."""
    tt = tau(t)
    return float(np.max(tt * users_xperp + users_y)), float(np.min(-tt * users_xperp + users_y))


def _trapezoid(x_min, x_max, y_min, y_max, t):
    tt = tau(t)
    L1 = x_min * tt + y_min
    R1 = min(x_min * tt + y_max, x_max * tt + y_min)
    L2 = max(x_min * tt + y_max, x_max * tt + y_min)
    R2 = x_max * tt + y_max
    return L1, R1, L2, R2


def expected_y_up_eq17(x_min, x_max, y_min, y_max, t, k):
    """eq. (17) with the (2K+1) reading of its fourth term."""
    L1, R1, L2, R2 = _trapezoid(x_min, x_max, y_min, y_max, t)
    q = (L2 - 2.0 * R1 + R2) / (2.0 * (R2 - R1))
    p = (R1 - L1) / (2.0 * (R2 - R1))
    inc_beta = special.betainc(1.5, k, p) * special.beta(1.5, k)
    return (R2
            - q ** k * (L2 - 2.0 * R1 + R2) / (2.0 * (k + 1))
            - q ** k * (R1 - L1)
            - p ** k * (R1 - L1) / (2.0 * (k + 1) * (2 * k + 1))
            - math.sqrt(2.0) * k * math.sqrt((R1 - L1) * (R2 - R1)) * inc_beta)


def expected_y_down_eq18(x_min, x_max, y_min, y_max, t, k):
    return y_min + y_max - expected_y_up_eq17(x_min, x_max, y_min, y_max, t, k)


def limit_y_up_eq19(x_max, y_max, t):
    return x_max * tau(t) + y_max


def limit_y_down_eq20(x_max, y_min, t):
    return y_min - x_max * tau(t)


def appendix_b_pdf_cdf(x_min, x_max, y_min, y_max, t):
    """Trapezoidal pdf and CDF of z_i (Appendix B)."""
    L1, R1, L2, R2 = _trapezoid(x_min, x_max, y_min, y_max, t)
    D1 = L2 - R1 + R2 - L1
    D2 = R1 - L1

    def pdf(z):
        if L1 <= z < R1:
            return 2.0 / D1 / D2 * (z - L1)
        if R1 <= z < L2:
            return 2.0 / D1
        if L2 <= z <= R2:
            return (R2 - z) * 2.0 / D1 / D2
        return 0.0

    def cdf(z):
        if z < L1:
            return 0.0
        if z < R1:
            return (z - L1) ** 2 / (D1 * D2)
        if z < L2:
            return (R1 - L1) / D1 + 2.0 / D1 * (z - R1)
        if z < R2:
            return 1.0 - (z - R2) ** 2 / (D1 * D2)
        return 1.0

    return pdf, cdf, (L1, R1, L2, R2)


def expected_y_up_appendix_b(x_min, x_max, y_min, y_max, t, k):
    """E[y_up] = int y K F(y)^{K-1} f(y) dy by adaptive quadrature (Appendix B)."""
    pdf, cdf, (L1, R1, L2, R2) = appendix_b_pdf_cdf(x_min, x_max, y_min, y_max, t)
    val, _ = integrate.quad(lambda y: y * k * cdf(y) ** (k - 1) * pdf(y), L1, R2,
                            points=[R1, L2], epsabs=1e-12, epsrel=1e-12, limit=400)
    return val


def saturation_m(e_up, e_down, spacing):
    """Antenna count spanned by [E y_down, E y_up] on a ULA of the given spacing."""
    return (e_up - e_down) / spacing


def empirical_saturation(n_list, cap, eps):
    """First N (log-interpolated) with cap(N) / cap(N_max) >= 1 - eps."""
    n_list = np.asarray(n_list, np.float64)
    c = np.asarray(cap, np.float64) / float(cap[-1])
    target = 1.0 - eps
    for i in range(len(c)):
        if c[i] >= target:
            if i == 0:
                return float(n_list[0])
            f = (target - c[i - 1]) / (c[i] - c[i - 1])
            return float(math.exp(math.log(n_list[i - 1]) + f * (math.log(n_list[i]) - math.log(n_list[i - 1]))))
    return float(n_list[-1])
