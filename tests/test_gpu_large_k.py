"""Drops with more users than one exact-Gram work item holds (K > 64, up to 1024).

The exact Gram runs such drops as one virtual drop per pair of user groups
(at most 32 users a group) and copies the blocks back; the sum-rates run one
workgroup per drop with the matrix in a global workspace.  Both against the
FP64 oracle, with the tolerances of the K <= 64 parity tests (normwise 1e-9
for the FP64 Gram, 1e-5 for FP32C/FP32H, 1e-9 relative for the rates).
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import channel as och
from oracle import rates as orates

pytestmark = pytest.mark.gpu

TOL = {"FP64": 1e-9, "FP32C": 1e-5, "FP32H": 1e-5}


@pytest.fixture(scope="module")
def X():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2503_18118_amd import xlmimo
    return xlmimo


@pytest.fixture(scope="module")
def ctx(X):
    c = X.Context(0)
    yield c
    c.close()


def _drops(ns, ks, seed, r=(2.0, 40.0), th=(-70.0, 70.0), z=False):
    rng = np.random.default_rng(seed)
    pos = []
    for k in ks:
        rr = rng.uniform(*r, k)
        t = np.deg2rad(rng.uniform(*th, k))
        zz = rng.uniform(-0.5, 0.5, k) if z else np.zeros(k)
        pos.append(np.stack([rr * np.cos(t), rr * np.sin(t), zz], axis=-1))
    return W._pack(ns, ks, np.concatenate(pos))


def _oracle_gram(arr, drops, d):
    a = arr.with_n(int(drops.n_elems[d])) if arr.geometry == W.GEOM_ULA else arr
    return och.gram_exact(a, drops.users_of(d))


@pytest.mark.parametrize("precision", ["FP64", "FP32C", "FP32H"])
def test_exact_large_k_ula(X, ctx, precision):
    # K = 65 (3 groups of 21-22), 100 (4 x 25), 130 (5 x 26), 200 (7 groups of 28-29),
    # 1024 (32 x 32, N < K) beside drops that fit one work item; N with ragged tails.
    ks = [65, 3, 100, 130, 64, 200, 1024, 1]
    ns = [300, 1000, 4097, 2000, 777, 3000, 257, 5]
    drops = _drops(ns, ks, seed=41)
    arr = W.ula(1, W.LAMBDA_28GHZ)
    b = X.Batch(drops)
    out = ctx.gram_exact(arr, b, getattr(X, precision))
    torch.cuda.synchronize()
    g = b.split(out)
    for d in range(drops.n_drops):
        ref = _oracle_gram(arr, drops, d)
        err = och.normwise_error(g[d], ref)
        assert err < TOL[precision], (precision, d, ns[d], ks[d], err)
        assert np.array_equal(g[d], g[d].conj().T)
    # the same drops one at a time give the same bits (the grouping depends on K only)
    for d in (0, 5):
        b1 = X.Batch(drops.subset([d]))
        g1 = b1.split(ctx.gram_exact(arr, b1, getattr(X, precision)))[0]
        assert np.array_equal(g1, g[d]), (precision, d)


@pytest.mark.parametrize("amp", [W.AMP_FREESPACE, W.AMP_PNUSW])
def test_exact_large_k_upa(X, ctx, amp):
    arr = W.ArraySpec(W.GEOM_UPA, 24, 20, 1.5e-3, 3.0e-3, amp)
    ks = [70, 5, 97]
    drops = _drops([arr.n_elems] * 3, ks, seed=43, r=(0.5, 3.0), z=True)
    b = X.Batch(drops)
    for precision in ("FP64", "FP32H"):
        g = b.split(ctx.gram_exact(arr, b, getattr(X, precision)))
        for d in range(drops.n_drops):
            err = och.normwise_error(g[d], _oracle_gram(arr, drops, d))
            assert err < TOL[precision], (amp, precision, d, err)


def _rho(rng, b, gh, n_snr):
    scale = 1e4 / np.mean([np.real(np.diag(m)).mean() for m in gh])
    return torch.as_tensor(rng.uniform(0.5, 2.0, (n_snr, b.total_users)) * scale, device="cuda")


def test_rates_large_k(X, ctx):
    # the workgroup-per-drop kernel runs the whole batch once any K > 64,
    # K <= 64 drops included
    ks = [70, 5, 129, 300, 64]
    ns = [4 * k + 300 for k in ks]
    drops = _drops(ns, ks, seed=47, r=(1.0, 6.0))
    arr = W.ula(1, W.LAMBDA_28GHZ)
    b = X.Batch(drops)
    g = ctx.gram_exact(arr, b, X.FP64)
    gh = b.split(g)
    rng = np.random.default_rng(5)
    rho = _rho(rng, b, gh, 2)
    names = [("ZF", orates.SCHEME_ZF), ("MMSE", orates.SCHEME_MMSE), ("MRC", orates.SCHEME_MRC),
             ("CAP", orates.SCHEME_CAP), ("CORR_GAP", orates.SCHEME_CORR_GAP)]
    rh = rho.cpu().numpy()
    for pick in (names, names[1:2], [names[3], names[4]], [names[0], names[2]]):
        schemes = sum(getattr(X, n) for n, _ in pick)
        rates, status = ctx.sumrate(b, g, rho, schemes)
        torch.cuda.synchronize()
        assert torch.all(status == 0)
        rates = rates.cpu().numpy()
        for d in range(drops.n_drops):
            for s in range(2):
                rk = rh[s, drops.user_off[d]:drops.user_off[d + 1]]
                ref = orates.rates(gh[d], rk, sum(key for _, key in pick))
                for c, (n, key) in enumerate(pick):
                    assert rates[d, s, c] == pytest.approx(ref[key], rel=1e-9), (n, d, ks[d], s)


def test_rates_large_k_not_pd(X, ctx):
    # a Gram with a negative diagonal entry: G and I + A are not positive definite
    ks = [80, 66]
    drops = _drops([600, 600], ks, seed=53, r=(1.0, 6.0))
    arr = W.ula(1, W.LAMBDA_28GHZ)
    b = X.Batch(drops)
    gh = b.split(ctx.gram_exact(arr, b, X.FP64))
    gh[0][3, 3] = -np.real(gh[0][3, 3])
    flat = torch.as_tensor(np.concatenate([m.ravel() for m in gh]).view(np.float64), device="cuda")
    rho = _rho(np.random.default_rng(1), b, gh, 1)
    rates, status = ctx.sumrate(b, flat, rho, X.ZF | X.MMSE | X.CAP | X.CORR_GAP)
    torch.cuda.synchronize()
    rates, status = rates.cpu().numpy(), status.cpu().numpy()
    assert status[0] == (X.ST_G_NOT_PD | X.ST_MMSE_NOT_PD) and status[1] == 0
    assert np.all(np.isnan(rates[0]))
    assert np.all(np.isfinite(rates[1]))


def test_large_k_limits(X, ctx):
    drops = _drops([400], [70], seed=59)
    arr = W.ula(1, W.LAMBDA_28GHZ)
    b = X.Batch(drops)
    g = ctx.gram_exact(arr, b, X.FP64)
    rho = torch.ones((1, b.total_users), dtype=torch.float64, device="cuda")
    with pytest.raises(X.XlmimoError, match="modified-ZF"):
        ctx.sumrate(b, g, rho, X.ZF | X.MZF, gram_filter=g)
    with pytest.raises(X.XlmimoError, match=r"outside 1\.\.64"):
        ctx.gram_closedform(arr, b, X.CF_PAPER)
    with pytest.raises(X.XlmimoError, match=r"outside 1\.\.64"):
        ctx.capacity_sweep(arr, [256, 512], b, X.FORM_CF_PAPER, rho, X.ZF)
    big = X.Batch(_drops([64], [X.MAX_USERS_EXACT + 1], seed=61))
    with pytest.raises(X.XlmimoError, match=r"outside 1\.\.1024"):
        ctx.gram_exact(arr, big, X.FP64)


def test_sweep_exact_large_k(X, ctx):
    # the exact sweep with K = 100 (the paper's Fig. 3 user count): ergodic
    # means over drops of the oracle's rates on the oracle's Grams
    arr = W.ula(1, W.LAMBDA_100GHZ, W.AMP_PNUSW)
    drops = W.rect_drops(W.rng_for(10, 3), 3, 100, 1, (1.0, 10.0), (-7.5, 7.5))
    b = X.Batch(drops)
    n_list = [2048, 8192]   # N = 512 leaves one drop with cond(G) ~ 3e5
    rho = torch.full((2, b.total_users), 1.0, dtype=torch.float64, device="cuda")
    rho[1] *= 1e3
    schemes = X.ZF | X.MMSE | X.CAP | X.CORR_GAP
    erg, sat, st = ctx.capacity_sweep(arr, n_list, b, X.FORM_EXACT_FP64, rho, schemes)
    torch.cuda.synchronize()
    erg = erg.cpu().numpy()
    assert torch.all(st == 0)
    keys = [orates.SCHEME_ZF, orates.SCHEME_MMSE, orates.SCHEME_CAP, orates.SCHEME_CORR_GAP]
    rh = rho.cpu().numpy()
    for i, n in enumerate(n_list):
        ref = np.zeros((2, 4))
        for d in range(drops.n_drops):
            gd = och.gram_exact(arr.with_n(n), drops.users_of(d))
            for s in range(2):
                r = orates.rates(gd, rh[s, drops.user_off[d]:drops.user_off[d + 1]], sum(keys))
                ref[s] += [r[k] for k in keys]
        ref /= drops.n_drops
        np.testing.assert_allclose(erg[i], ref, rtol=1e-8, atol=0)
