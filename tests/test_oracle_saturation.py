"""Pins of the saturation analysis (Sec. IV, Appendices B-C): eq. (12) against
eq. (11), eq. (17) against the Appendix B integral and Monte Carlo, eq. (18)
symmetry, eqs. (19)-(20) limits, and the values the paper prints."""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import saturation as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def test_eq12_solves_eq11():
    lam = W.LAMBDA_100GHZ
    for x, t in [(1.5, 0.9), (4.0, 0.5), (10.0, 0.99)]:
        m = S.m_single_user_eq12(x, t, lam)
        assert S.power_ratio_eq11(x, 0.0, m, lam) == pytest.approx(t, rel=1e-12)
        # and the array then spans [-tau x, tau x] (text after eq. (12))
        assert m * lam / 4 == pytest.approx(S.tau(t) * x, rel=1e-12)


@pytest.mark.parametrize("k", [1, 2, 10, 100, 1000])
@pytest.mark.parametrize("scene", [(1.0, 10.0, -7.5, 7.5), (1.0, 2.0, -7.5, 7.5), (2.0, 3.0, -0.5, 0.5)])
def test_eq17_equals_appendix_b_integral(k, scene):
    xmin, xmax, ymin, ymax = scene
    a = S.expected_y_up_eq17(xmin, xmax, ymin, ymax, 0.9, k)
    b = S.expected_y_up_appendix_b(xmin, xmax, ymin, ymax, 0.9, k)
    assert a == pytest.approx(b, rel=1e-9, abs=1e-9)


def test_eq17_eq18_vs_monte_carlo():
    rng = np.random.default_rng(11)
    t, k = 0.9, 10
    xmin, xmax, ymin, ymax = 1.0, 2.0, -7.5, 7.5
    n = 200_000
    x = rng.uniform(xmin, xmax, (n, k))
    y = rng.uniform(ymin, ymax, (n, k))
    tt = S.tau(t)
    up = np.max(tt * x + y, axis=1)
    dn = np.min(-tt * x + y, axis=1)
    e_up = S.expected_y_up_eq17(xmin, xmax, ymin, ymax, t, k)
    e_dn = S.expected_y_down_eq18(xmin, xmax, ymin, ymax, t, k)
    assert abs(up.mean() - e_up) < 4 * up.std() / math.sqrt(n)
    assert abs(dn.mean() - e_dn) < 4 * dn.std() / math.sqrt(n)


def test_eq19_eq20_limits():
    t = 0.9
    a = S.expected_y_up_eq17(1.0, 10.0, -7.5, 7.5, t, 10 ** 9)
    assert a == pytest.approx(S.limit_y_up_eq19(10.0, 7.5, t), rel=1e-4)
    b = S.expected_y_down_eq18(1.0, 10.0, -7.5, 7.5, t, 10 ** 9)
    assert b == pytest.approx(S.limit_y_down_eq20(10.0, -7.5, t), rel=1e-4)
    # Appendix C: the remaining gap is dominated by the incomplete-beta term, O(K^{-1/2})
    lim = S.limit_y_up_eq19(10.0, 7.5, t)
    g1 = lim - S.expected_y_up_eq17(1.0, 10.0, -7.5, 7.5, t, 10 ** 4)
    g4 = lim - S.expected_y_up_eq17(1.0, 10.0, -7.5, 7.5, t, 4 * 10 ** 4)
    assert g4 / g1 == pytest.approx(0.5, rel=0.01)
    # monotone approach (Sec. IV-B: terms rise to their limit 0 with K)
    vals = [S.expected_y_up_eq17(1.0, 10.0, -7.5, 7.5, t, k) for k in (1, 2, 5, 10, 100, 1000)]
    assert all(v1 < v2 for v1, v2 in zip(vals, vals[1:]))


def test_paper_printed_values():
    with open(GOLDEN) as f:
        gold = json.load(f)
    sec5 = gold["sec5_saturation_antennas"]
    e_up = S.expected_y_up_eq17(1.0, 2.0, -7.5, 7.5, 0.9, 10)
    e_dn = S.expected_y_down_eq18(1.0, 2.0, -7.5, 7.5, 0.9, 10)
    m = S.saturation_m(e_up, e_dn, W.LAMBDA_100GHZ / 2)
    # the paper gives the saturation scale as about ten thousand antennas: same order of magnitude
    assert sec5["value"] / 2 < m < sec5["value"] * 2
    # Appendix A's packing arithmetic as printed (a consistency check of the golden values,
    # not a pin of an oracle function): 2 / (sqrt 3 d^2) ~= 4.619 users/m^2, K <= ~693
    dens = gold["hexagonal_density_per_m2"]
    d = dens["spacing_m"]
    assert 2 / (math.sqrt(3) * d * d) == pytest.approx(dens["value"], abs=5e-4)
    assert 15 * 10 * dens["value"] == pytest.approx(gold["user_cap"]["value"], abs=0.5)


def test_y_bounds_hand_drop():
    # eqs. (13)-(16) by hand at t = 0.6, tau = 0.6 / 0.8 = 0.75:
    # users (2, 1), (4, -1), (1, 3) give y_up^i = 2.5, 2.0, 3.75 and y_down^i = -0.5, -4.0, 2.25
    x = np.array([2.0, 4.0, 1.0])
    y = np.array([1.0, -1.0, 3.0])
    up, dn = S.y_bounds_eq15_16(x, y, 0.6)
    assert up == pytest.approx(3.75, rel=1e-15)
    assert dn == pytest.approx(-4.0, rel=1e-15)
    # the user that sets each bound: the last one for y_up, the second for y_down
    assert S.y_bounds_eq15_16(x[[0, 1]], y[[0, 1]], 0.6)[0] == pytest.approx(2.5, rel=1e-15)
    assert S.y_bounds_eq15_16(x[[0, 2]], y[[0, 2]], 0.6)[1] == pytest.approx(-0.5, rel=1e-15)


@pytest.mark.parametrize("x,t", [(1.5, 0.9), (4.0, 0.5), (10.0, 0.99)])
def test_y_bounds_single_user_is_eq12(x, t):
    # one user at y = 0: the bounds are +-tau x (text after eq. (12)), and the ULA of
    # half-wavelength spacing that spans them has the eq. (12) antenna count
    lam = W.LAMBDA_100GHZ
    up, dn = S.y_bounds_eq15_16(np.array([x]), np.array([0.0]), t)
    assert up == pytest.approx(-dn, rel=1e-15)
    assert S.saturation_m(up, dn, lam / 2) == pytest.approx(S.m_single_user_eq12(x, t, lam), rel=1e-12)
    # a user off centre shifts both bounds by its y (eqs. (13)-(14))
    up2, dn2 = S.y_bounds_eq15_16(np.array([x]), np.array([2.5]), t)
    assert up2 - up == pytest.approx(2.5, rel=1e-12) and dn2 - dn == pytest.approx(2.5, rel=1e-12)


def test_y_bounds_mean_matches_eq17_eq18():
    # the mean of eqs. (15)-(16) over the Sec. V scene's drops (x ~ U(1,2) m, y ~ U[-7.5,7.5] m,
    # K = 10, t = 0.9) converges to eqs. (17)-(18); 10^5 drops, within 4 standard errors
    arr, drops, meta = W.paper_sec5(n_drops=100_000)
    t = meta["t"]
    ups = np.empty(drops.n_drops)
    dns = np.empty(drops.n_drops)
    for d in range(drops.n_drops):
        u = drops.users_of(d)
        ups[d], dns[d] = S.y_bounds_eq15_16(u[:, 0], u[:, 1], t)
    n = drops.n_drops
    e_up = S.expected_y_up_eq17(1.0, 2.0, -7.5, 7.5, t, 10)
    e_dn = S.expected_y_down_eq18(1.0, 2.0, -7.5, 7.5, t, 10)
    assert abs(ups.mean() - e_up) < 4 * ups.std() / math.sqrt(n)
    assert abs(dns.mean() - e_dn) < 4 * dns.std() / math.sqrt(n)
    # and the saturation antenna count of the paper's Sec. V-C statement follows from them
    m_mc = S.saturation_m(ups.mean(), dns.mean(), W.LAMBDA_100GHZ / 2)
    m_cf = S.saturation_m(e_up, e_dn, W.LAMBDA_100GHZ / 2)
    assert m_mc == pytest.approx(m_cf, rel=2e-3)


def test_empirical_saturation_interpolates():
    n = [256, 1024, 4096, 16384]
    cap = [50.0, 80.0, 95.0, 100.0]
    # 0.9 lies between 0.8 (N=1024) and 0.95 (N=4096): 2/3 of the way in log N
    want = math.exp(math.log(1024) + (0.9 - 0.8) / 0.15 * math.log(4))
    assert S.empirical_saturation(n, cap, 0.1) == pytest.approx(want, rel=1e-12)
    assert S.empirical_saturation(n, cap, 0.6) == 256
