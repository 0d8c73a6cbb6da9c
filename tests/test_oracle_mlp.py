"""Pins of the FP64 MLP reference: finite-difference gradients, GELU's erf form,
Adam on a quadratic, and the phasor basis against the exact channel phases."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import channel as och
from oracle import closedform as ocf
from oracle import mlp as M


def _batch(rng, n):
    x = rng.normal(size=(n, M.N_IN))
    ph = np.exp(1j * rng.uniform(-math.pi, math.pi, size=(n, 3)))
    t = 0.05 * (rng.normal(size=n) + 1j * rng.normal(size=n))
    return x, ph, t


def test_gelu_matches_closed_form_values():
    # GELU(z) = z Phi(z): Phi(1) = 0.841344746..., Phi(-1) = 0.158655253...
    assert M.gelu(np.array([1.0]))[0] == pytest.approx(0.8413447460685429, rel=1e-14)
    assert M.gelu(np.array([-1.0]))[0] == pytest.approx(-0.15865525393145707, rel=1e-14)
    z = np.linspace(-4, 4, 41)
    h = 1e-6
    assert np.allclose(M.gelu_grad(z), (M.gelu(z + h) - M.gelu(z - h)) / (2 * h), rtol=1e-8, atol=1e-10)


@pytest.mark.parametrize("width,depth", [(8, 2), (16, 4)])
def test_gradient_matches_finite_differences(width, depth):
    rng = np.random.default_rng(1)
    p = M.init_params(rng, width, depth)
    p[-M.N_OUT:] = rng.normal(size=M.N_OUT) * 0.1   # non-trivial output bias
    x, ph, t = _batch(rng, 37)
    loss, g = M.loss_grad(p, x, ph, t, width, depth)
    idx = rng.choice(p.size, 40, replace=False)
    for i in idx:
        e = np.zeros_like(p)
        h = 1e-6 * max(1.0, abs(p[i]))
        e[i] = h
        fd = (M.loss_grad(p + e, x, ph, t, width, depth)[0] - M.loss_grad(p - e, x, ph, t, width, depth)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-6, abs=1e-9), i


def test_adam_converges_on_quadratic():
    rng = np.random.default_rng(2)
    target = rng.normal(size=10)
    w = np.zeros(10)
    opt = M.Adam(10, lr=0.05)
    for _ in range(3000):
        w = opt.step(w, w - target)
    assert np.allclose(w, target, atol=1e-4)
    # first step of Adam moves every coordinate by lr (bias-corrected m/sqrt(v) = sign(g))
    opt = M.Adam(3, lr=0.1)
    assert np.allclose(opt.step(np.zeros(3), np.array([2.0, -5.0, 0.3])), [-0.1, 0.1, -0.1], atol=1e-6)


def test_param_layout():
    assert M.param_count(256, 4) == 6 * 256 + 256 + 3 * (256 * 256 + 256) + 256 * 7 + 7
    p = np.arange(M.param_count(4, 2), dtype=float)
    (w0, b0), (w1, b1), (w2, b2) = M.unpack(p, 4, 2)
    assert w0.shape == (4, 6) and b0[0] == 24 and w2.shape == (7, 4)


def test_basis_phases_and_end_correction():
    # the end terms carry the exact channel phase of conj(h_i) h_j at the end elements, and
    # with c_top = c_bot = 1 they remove most of the closed form's error (the discrete sum's
    # end contributions): pinned against the exact Gram of the channel oracle
    lam = W.LAMBDA_28GHZ
    n = 4096
    arr = W.ula(n, lam)
    rng = np.random.default_rng(4)
    errs_cf, errs_end = [], []
    for _ in range(30):
        r = rng.uniform(5, 50, 2)
        th = np.deg2rad(rng.uniform(-60, 60, 2))
        u = np.stack([r * np.cos(th), r * np.sin(th), np.zeros(2)], axis=-1)
        g = och.gram_exact(arr, u)
        gc = ocf.gram_closedform(arr, u, n, ocf.VARIANT_GATED)
        sc = math.sqrt(gc[0, 0].real * gc[1, 1].real)
        f, b = M.pair_inputs(u[0, 0], u[0, 1], u[1, 0], u[1, 1], n, arr.spacing, lam, sc)
        ref = math.sqrt(g[0, 0].real * g[1, 1].real)
        errs_cf.append(abs(gc[0, 1] - g[0, 1]) / ref)
        errs_end.append(abs(gc[0, 1] + (b[0] + b[1]) * sc - g[0, 1]) / ref)
    assert np.median(errs_end) < 1e-3 * np.median(errs_cf)
    assert f[4] == pytest.approx(math.log(4096) / math.log(4) - 6)


def test_basis_end_term_matches_geometric_series():
    # far from phi' = 0 the regularisation is negligible and b_top * cf_scale equals the
    # geometric series f e^{j phi} / (1 - e^{-j phi' d}) evaluated from the channel itself
    lam = W.LAMBDA_28GHZ
    n = 1024
    arr = W.ula(n, lam)
    u = np.array([[3.0, -2.0, 0.0], [9.0, 4.0, 0.0]])
    h = och.channel_matrix(arr, u)
    p_end = h[-1, 0].conj() * h[-1, 1]
    p_prev = h[-2, 0].conj() * h[-2, 1]
    ratio = p_prev / p_end                    # ~ e^{-j phi' d} |...| for the locally linear phase
    series = p_end / (1 - ratio / abs(ratio))
    f, b = M.pair_inputs(3.0, -2.0, 9.0, 4.0, n, arr.spacing, lam, 1.0)
    assert abs(b[0] - series) < 2e-2 * abs(series)
    # the stationary-point phasor carries the eq. (6) phase before the -pi/4 offset
    rho = ocf.rho_eq6(3.0, -2.0, 9.0, 4.0, n, lam)
    assert abs(b[2] * np.exp(-1j * math.copysign(1, 3.0 - 9.0) * math.pi / 4) - rho / abs(rho)) < 1e-9


def test_basis_end_term_is_bounded_where_phase_is_stationary():
    # users on one ray leaving the top element make phi'(y_top) = 0: the geometric series
    # would diverge; the regularised term is bounded by f / (2 eps), eps = d sqrt(|phi''| / 2 pi),
    # and vanishes at the singular point itself
    lam = W.LAMBDA_28GHZ
    n = 2001
    d = lam / 2
    yt = (n - 1) * d / 2
    ang = math.radians(30)
    k = 2 * math.pi / lam
    for shift in (0.0, 1e-4, 1e-3, 1e-2):
        xi, yi = 4 * math.cos(ang), yt - 4 * math.sin(ang) + shift
        xj, yj = 9 * math.cos(ang), yt - 9 * math.sin(ang)
        f, b = M.pair_inputs(xi, yi, xj, yj, n, d, lam, 1.0)
        a, bb = math.hypot(xi, yt - yi), math.hypot(xj, yt - yj)
        amp = (lam / (4 * math.pi)) ** 2 / (a * bb)
        d2 = k * (xi ** 2 / a ** 3 - xj ** 2 / bb ** 3)
        eps = d * math.sqrt(abs(d2) / (2 * math.pi))
        assert abs(b[0]) <= amp / (2 * eps) * (1 + 1e-9)
        if shift == 0.0:
            assert abs(b[0]) < 1e-6 * amp / (2 * eps)


def test_loss_is_minimised_by_the_target():
    rng = np.random.default_rng(3)
    x, ph, t = _batch(rng, 50)
    out = np.zeros((50, 7))
    # choose c_top so that p = t exactly (c_bot = 0: its output cancels the analytic C0 = 1);
    # s = 0 and e = 0 give loss = 0
    out[:, 0] = (t * ph[:, 0].conj()).real - 1.0
    out[:, 1] = (t * ph[:, 0].conj()).imag
    out[:, 2] = -1.0
    p, s = M.predict(out, ph)
    assert np.allclose(p, t)
    loss, dout = M.loss_and_dout(out, ph, t)
    assert loss == pytest.approx(0.0)
    assert np.allclose(dout[:, :6], 0.0)


def test_basis_is_zero_for_slow_phase_pairs():
    # users a few centimetres apart have no stationary-phase regime: the base closed form integrates
    # them (variant GATED_QUAD) and the network gets a zero basis there
    lam = W.LAMBDA_28GHZ
    arr = W.ula(4096, lam)
    f, b = M.pair_inputs(9.0, 1.0, 9.03, 1.02, 4096, arr.spacing, lam, 1.0)
    assert np.all(b == 0)
    assert ocf.slow_pair_panels(arr, 9.0, 1.0, 9.03, 1.02, 4096) > 0
    f, b = M.pair_inputs(9.0, 1.0, 20.0, 7.0, 4096, arr.spacing, lam, 1.0)
    assert np.all(b != 0) and ocf.slow_pair_panels(arr, 9.0, 1.0, 20.0, 7.0, 4096) == 0
