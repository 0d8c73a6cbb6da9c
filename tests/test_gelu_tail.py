"""The GELU forward of the network kernels, evaluated on the CPU in float32.

The kernels take GELU(z) = max(z, 0) - |z| 2^P(min(|z|, 6)), P a degree-6
polynomial fitted to log2 of the Gaussian tail erfc(x / sqrt 2) / 2.  The
coefficients are read from the kernel source, so a mistyped constant fails here:
the float32 evaluation (Horner, exp2, the final FMA) must stay within 3e-7 of the
oracle's erf-form GELU (1.6e-7 relative near zero, where P(0) = -1 makes
GELU(z) ~ z / 2 exact), and the fit must reproduce the constants.
"""
import os
import re

import numpy as np

from oracle import mlp as omlp
from paper_2503_18118_amd import fit_gelu_tail

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_2503_18118_amd", "csrc", "mlp.hip")


def kernel_coefficients():
    src = open(SRC).read()
    body = src[src.index("__device__ __forceinline__ float gelu(float z)"):]
    body = body[:body.index("\n}\n")]
    vals = [float(v) for v in re.findall(r"([-+]?\d\.\d+e[-+]\d+)f", body)]
    assert len(vals) == 7, vals
    # written from the top coefficient down: x^6, x^5, x^4, ..., x^0
    return np.array(vals[::-1])


def test_kernel_gelu_matches_erf_form():
    c = kernel_coefficients()
    z = np.linspace(-30.0, 30.0, 600001).astype(np.float32)
    got = fit_gelu_tail.gelu_f32(z, c).astype(np.float64)
    ref = omlp.gelu(z.astype(np.float64))
    err = np.abs(got - ref)
    assert err.max() <= 3.2e-7, err.max()
    # small |z|: GELU ~ z / 2, the error stays relative-small too
    small = np.abs(z) < 1e-2
    assert np.all(err[small] <= 2e-7 * np.abs(z[small])), (err[small] / np.abs(z[small] + 1e-30)).max()


def test_fit_reproduces_kernel_constants():
    c = fit_gelu_tail.fit()
    np.testing.assert_allclose(kernel_coefficients(), c, rtol=1e-8, atol=0)
