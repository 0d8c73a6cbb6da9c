"""Coefficients of the GELU forward used by the network kernels (``csrc/mlp.hip``).

GELU(z) = z Phi(z) = max(z, 0) - |z| Q(|z|), with Q(x) = erfc(x / sqrt 2) / 2 the
Gaussian tail.  The kernels take Q(x) = 2^P(x), P a polynomial of degree 6 in
x = min(|z|, X), X = 6, with P(0) = -1 (Q(0) = 1/2 exactly, so GELU(z) ~ z / 2 keeps
its relative accuracy near zero): P(x) = -1 + x R(x), R of degree 5 fitted to
(log2 Q(x) + 1) / x on (0, X] by iteratively reweighted least squares on the error
of x Q(x), the term GELU subtracts (an error e in R moves it by x^2 Q(x) ln2 e).
Run as ``python -m paper_2503_18118_amd.fit_gelu_tail``; it prints the coefficients
and the largest GELU error of the polynomial evaluated in float32 (Horner, exp2 of
the result), over [-30, 30].
"""
import numpy as np
from scipy.special import erfc

X = 6.0
DEGREE = 6


def tail(x):
    return 0.5 * erfc(x / np.sqrt(2.0))


def fit(x_max=X, degree=DEGREE, passes=40):
    """Coefficients of P, x^0 .. x^degree, with P(0) = -1."""
    xs = np.linspace(0.0, x_max, 200001)[1:]
    q = tail(xs)
    target = (np.log2(q) + 1.0) / xs
    weight = xs * xs * q * np.log(2.0) + 1e-12
    w = weight.copy()
    for _ in range(passes):
        r = np.polynomial.polynomial.polyfit(xs, target, degree - 1, w=w)
        err = np.abs(np.polynomial.polynomial.polyval(xs, r) - target) * weight
        w = w * (1.0 + 5.0 * err / err.max())
    return np.concatenate([[-1.0], r])


def gelu_f32(z, c, x_max=X):
    f = np.float32
    zf = np.asarray(z, dtype=f)
    x = np.minimum(np.abs(zf), f(x_max))
    p = f(c[-1])
    for k in range(len(c) - 2, -1, -1):
        p = (p * x + f(c[k])).astype(f)
    q = np.exp2(p.astype(np.float64)).astype(f)
    return (-np.abs(zf) * q + np.maximum(zf, f(0))).astype(f)


if __name__ == "__main__":
    c = fit()
    z = np.linspace(-30.0, 30.0, 600001).astype(np.float32)
    zd = z.astype(np.float64)
    exact = zd * 0.5 * erfc(-zd / np.sqrt(2.0))
    print("P coefficients, x^0 .. x^6:", ", ".join(f"{v:.9e}" for v in c))
    print("max |GELU error| in float32:", float(np.abs(gelu_f32(z, c) - exact).max()))
