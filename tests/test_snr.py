"""The SNR convention of the workloads (paper_2503_18118_amd/snr.py) against the oracle.

The reference gain of a ULA is the N -> infinity limit of a broadside user's Gram
diagonal: pinned here against the exact diagonal of the channel oracle at growing N
(free space) and against eq. (5) (PNUSW).  No GPU is used."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import channel as och
from oracle import closedform as ocf
from paper_2503_18118_amd import snr


def test_free_space_reference_gain_is_the_diagonal_limit():
    lam = W.LAMBDA_28GHZ
    x = 27.5
    g_ref = snr.reference_gain(W.ula(1, lam), x)
    assert g_ref == pytest.approx(lam / (8 * math.pi * x), rel=1e-14)   # d = lambda / 2
    u = np.array([[x, 0.0, 0.0]])
    prev = None
    for n in (65536, 262144, 1048576):
        g = och.gram_exact(W.ula(n, lam), u)[0, 0].real
        assert g < g_ref
        if prev is not None:        # the aperture's missing tail shrinks as 1/N
            assert (g_ref - g) < 0.3 * (g_ref - prev)
            g_inf = g + (g - prev) / 3.0    # Richardson step for a 1/N tail (N grows 4x)
        prev = g
    assert g_inf == pytest.approx(g_ref, rel=1e-4)


def test_pnusw_reference_gain_is_eq5():
    lam = W.LAMBDA_100GHZ
    arr = W.ula(1, lam, W.AMP_PNUSW)
    for x in (1.5, 5.5):
        assert snr.reference_gain(arr, x) == pytest.approx(ocf.power_limit_eq5(x, lam), rel=1e-12)


def test_rho_is_snr_over_gain_for_every_user():
    arr = W.ula(256, W.LAMBDA_28GHZ)
    rho = snr.rho_host(arr, (0.0, 10.0, 20.0), 27.5, 7)
    g = snr.reference_gain(arr, 27.5)
    assert rho.shape == (3, 7)
    assert np.allclose(rho * g, np.array([1.0, 10.0, 100.0])[:, None], rtol=1e-14)
