"""FP64 reference of the learned residual correction of the closed-form correlation.

Not part of the paper: the benchmark workload defines a small MLP that predicts
the residual rho_exact - rho~ of the closed-form correlation (eq. (6) and its
free-space analogue, eq. (23)) where stationary phase is inaccurate (small N,
users near the aperture ends; the paper notes the modified ZF is worse before
saturation, Sec. V-C).  Parity of the HIP kernels against this module is
pinned by finite differences (gradients), by the erf form of GELU, by Adam on a
quadratic, and by the exact channel phases at the aperture ends (phasors).

Pair inputs (user i, user j of one drop; x = perpendicular distance, y along the array):
  features  f = (r_i / 50, theta_i / (pi/3), r_j / 50, theta_j / (pi/3), log4(N) - 6, d/lambda - 1/2),
            r = sqrt(x^2 + y^2), theta = atan2(y, x) (polar coordinates about the array centre)
  basis     three complex terms in correlation units (divided by sqrt(G~_ii G~_jj)):
            b_top, b_bot = the end-element contributions of the discrete sum
              sum_n f(y_n) e^{j phi(y_n)}: locally linear phase at the end element y_e gives the
              geometric series f(y_e) e^{j phi(y_e)} / D, D = 1 - e^{-+ j phi'(y_e) d}
              (- at the top end y_top = (N-1) d/2, + at the bottom end y_bot = -y_top);
              1/D is regularised as conj(D) / (|D|^2 + eps^2) with the Fresnel scale
              eps = d sqrt(|phi''(y_e)| / (2 pi)): |b| never exceeds f / (2 eps) (reached at
              |D| = eps) and the term fades out where the phase becomes stationary at the end
              (D -> 0), the regime the network and the exact fallback handle;
            b_spm = e^{j phi(y*)}, y* the stationary point (y_i x_j - x_i y_j)/(x_j - x_i)
              (1 when x_i == x_j);
            phi(y) = (2 pi/lambda)(r_i(y) - r_j(y)), f = |h_i(y)| |h_j(y)| of the channel model;
            all three are 0 for a pair the base closed form (GATED_QUAD) evaluates numerically
            (closedform.numeric_route: slow-phase pairs and broad stationary zones).
  target    delta = rho_exact_ij - rho~_ij (complex)
Network: 6 -> [Linear(w) + GELU] x depth -> Linear(7); GELU(z) = z (1 + erf(z / sqrt 2)) / 2.
Output o: coefficients c_m = C0_m + o[2m] + j o[2m+1] (m = top, bot, star) and s = o[6] = log sigma^2,
  with C0 = (1, 1, 0): an all-zero output is the analytic end correction (both end terms of the
  discrete sum added to the closed form), and the network predicts how far the coefficients lie from it;
  prediction  p = sum_m c_m b_m
  loss        mean over pairs of |delta - p|^2 e^{-s} + s        (Gaussian negative log-likelihood)
Parameters, flat, layer by layer: W (out x in, row-major) then b (out).
Adam (Kingma & Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
  w -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special

from .closedform import ROUTE_NONE, numeric_route

N_IN = 6
N_OUT = 7
R_NORM = 50.0
THETA_NORM = math.pi / 3


def layer_shapes(width=256, depth=4):
    dims = [N_IN] + [width] * depth + [N_OUT]
    return [(dims[i + 1], dims[i]) for i in range(len(dims) - 1)]


def param_count(width=256, depth=4):
    return sum(o * i + o for o, i in layer_shapes(width, depth))


def unpack(params, width=256, depth=4):
    out, off = [], 0
    for o, i in layer_shapes(width, depth):
        w = params[off:off + o * i].reshape(o, i)
        off += o * i
        b = params[off:off + o]
        off += o
        out.append((w, b))
    assert off == params.size
    return out


def init_params(rng, width=256, depth=4):
    """He-normal weights, zero biases (the last layer scaled down by 1e-2)."""
    parts = []
    shapes = layer_shapes(width, depth)
    for li, (o, i) in enumerate(shapes):
        w = rng.normal(0.0, math.sqrt(2.0 / i), size=(o, i))
        if li == len(shapes) - 1:
            w *= 1e-2
        parts += [w.ravel(), np.zeros(o)]
    return np.concatenate(parts)


def gelu(z):
    return 0.5 * z * (1.0 + special.erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + special.erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def pair_inputs(xp_i, y_i, xp_j, y_j, n, spacing, lam, cf_scale, amp_model=0, beta0=1.0):
    """Features [6] and basis [3] (complex) of one pair; x are perpendicular distances,
    cf_scale = sqrt(G~_ii G~_jj) of the closed form."""
    k = 2.0 * math.pi / lam
    r_i, r_j = math.hypot(xp_i, y_i), math.hypot(xp_j, y_j)
    f = np.array([r_i / R_NORM, math.atan2(y_i, xp_i) / THETA_NORM, r_j / R_NORM,
                  math.atan2(y_j, xp_j) / THETA_NORM, math.log(n) / math.log(4.0) - 6.0, spacing / lam - 0.5])

    def dist(y):
        return math.hypot(xp_i, y - y_i), math.hypot(xp_j, y - y_j)

    def phi(y):
        a, b = dist(y)
        return k * (a - b)

    def amp(y):
        a, b = dist(y)
        if amp_model == 0:
            return (lam / (4.0 * math.pi)) ** 2 / (a * b)
        return beta0 * math.sqrt(xp_i * xp_j) / (a * b) ** 1.5

    def end_term(y, sign):
        a, b = dist(y)
        d1 = k * ((y - y_i) / a - (y - y_j) / b)
        d2 = k * (xp_i ** 2 / a ** 3 - xp_j ** 2 / b ** 3)
        den = 1.0 - np.exp(-1j * sign * d1 * spacing)
        eps2 = spacing ** 2 * abs(d2) / (2.0 * math.pi)
        return amp(y) * np.exp(1j * phi(y)) * np.conj(den) / (abs(den) ** 2 + eps2) / cf_scale

    y_top = (n - 1) * spacing / 2.0
    # pairs the base closed form evaluates numerically (GATED_QUAD, UNIFORM): no correction
    if numeric_route(spacing, lam, xp_i, y_i, xp_j, y_j, n)[0] != ROUTE_NONE:
        return f, np.zeros(3, np.complex128)
    if xp_i == xp_j:
        ps = 1.0 + 0j
    else:
        ys = (y_i * xp_j - xp_i * y_j) / (xp_j - xp_i)
        ps = np.exp(1j * phi(ys))
    return f, np.array([end_term(y_top, 1.0), end_term(-y_top, -1.0), ps])


def forward(params, x, width=256, depth=4):
    """x [n, 6] -> (out [n, 7], cache)."""
    layers = unpack(params, width, depth)
    a = x
    cache = []
    for li, (w, b) in enumerate(layers):
        z = a @ w.T + b
        cache.append((a, z))
        a = gelu(z) if li < len(layers) - 1 else z
    return a, cache


C0 = np.array([1.0, 1.0, 0.0])   # basis coefficients of the analytic end correction


def predict(out, phasors):
    """Complex prediction p [n] and log-variance s [n] from the network output."""
    c = C0 + out[:, 0:6:2] + 1j * out[:, 1:6:2]
    return np.sum(c * phasors, axis=1), out[:, 6]


def loss_and_dout(out, phasors, target):
    """Mean Gaussian NLL and its gradient with respect to the network output."""
    n = out.shape[0]
    p, s = predict(out, phasors)
    e = target - p
    w = np.exp(-s)
    loss = float(np.mean(np.abs(e) ** 2 * w + s))
    # dL/dp_r = -2 e_r w, dL/dp_i = -2 e_i w (per sample, then / n)
    gpr = -2.0 * e.real * w / n
    gpi = -2.0 * e.imag * w / n
    dout = np.zeros_like(out)
    for m in range(3):
        cph, sph = phasors[:, m].real, phasors[:, m].imag
        # p_r = sum a cos - b sin, p_i = sum a sin + b cos
        dout[:, 2 * m] = gpr * cph + gpi * sph
        dout[:, 2 * m + 1] = -gpr * sph + gpi * cph
    dout[:, 6] = (1.0 - np.abs(e) ** 2 * w) / n
    return loss, dout


def backward(params, cache, dout, width=256, depth=4):
    """Flat gradient of the loss with respect to the parameters."""
    layers = unpack(params, width, depth)
    grads = [None] * len(layers)
    d = dout
    for li in range(len(layers) - 1, -1, -1):
        a, z = cache[li]
        if li < len(layers) - 1:
            d = d * gelu_grad(z)
        w, _ = layers[li]
        grads[li] = (d.T @ a, d.sum(axis=0))
        d = d @ w
    return np.concatenate([np.concatenate([gw.ravel(), gb]) for gw, gb in grads])


def loss_grad(params, x, phasors, target, width=256, depth=4):
    out, cache = forward(params, x, width, depth)
    loss, dout = loss_and_dout(out, phasors, target)
    return loss, backward(params, cache, dout, width, depth)


class Adam:
    def __init__(self, n, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, params, g, lr=None):
        lr = self.lr if lr is None else lr
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return params - lr * mh / (np.sqrt(vh) + self.eps)
