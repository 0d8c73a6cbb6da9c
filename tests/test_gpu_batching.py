"""Batching: graph capture of library call sequences and the exact-Gram autotuner, through the C ABI.

A captured graph must replay exactly what the eager calls compute (bitwise: every
kernel has a fixed summation order), also after unrelated eager work between the
replays; an autotuned launch shape must keep the oracle parity of the exact Gram.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import channel as och
from oracle import mlp as OM

pytestmark = pytest.mark.gpu


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


def _sweep_setup(X):
    arr = W.ula(4096, W.LAMBDA_28GHZ)
    drops = W.polar_drops(W.rng_for(7), 48, 8, 4096, (5.0, 50.0), (-60.0, 60.0))
    b = X.Batch(drops)
    from paper_2503_18118_amd import snr
    rho = snr.rho_for_snr(arr, (0.0, 20.0), 27.5, b.total_users)
    return arr, drops, b, rho


def _outputs(b, n_n, n_snr, n_sch, dev):
    return (torch.empty((n_n, n_snr, n_sch), dtype=torch.float64, device=dev),
            torch.empty(3 + n_snr * n_sch, dtype=torch.float64, device=dev),
            torch.empty((n_n, b.n_drops), dtype=torch.int32, device=dev))


def test_graph_replays_match_eager(X, ctx):
    arr, drops, b, rho = _sweep_setup(X)
    n_list = [64, 256, 1024, 4096]
    schemes = X.ZF | X.MMSE
    dev = b.pos.device
    mlp = X.MLP(ctx, 64, 2)
    params = OM.init_params(np.random.default_rng(3), 64, 2)
    params[-1] = -30.0  # confident network: no fallback, the corrected Grams go straight to the rates
    mlp.set_params(params.astype(np.float32))
    s = torch.cuda.Stream()
    forms = [(X.FORM_EXACT_FP32H, {}), (X.FORM_CF_GATED, {}), (X.FORM_CF_UNIFORM, {}),
             (X.FORM_CF_GATED_MLP, {"mlp": mlp, "log_var_max": 0.0})]
    outs = [_outputs(b, len(n_list), 2, 2, dev) for _ in forms]
    gram = torch.empty(2 * b.gram_elems, dtype=torch.float64, device=dev)

    def run_all():
        for (form, kw), (e, sa, st) in zip(forms, outs):
            ctx.capacity_sweep(arr, n_list, b, form, rho, schemes, 0.9, 0.05, e, sa, st, stream=s, **kw)
        ctx.gram_exact(arr, b, X.FP32H, out=gram, stream=s)

    run_all()  # eager (and warm: plans, workspace, N list)
    s.synchronize()
    want = [tuple(t.clone() for t in o) for o in outs] + [gram.clone()]
    ctx.graph_begin(s)
    run_all()
    g = ctx.graph_end(s)
    assert g.n_nodes > 20
    other = X.Batch(W.polar_drops(W.rng_for(8), 5, 3, 300, (5.0, 50.0), (-60.0, 60.0)))
    for r in range(3):
        with torch.cuda.stream(s):
            for o in outs:
                for t in o:
                    t.fill_(-1)
            gram.fill_(-1)
        # unrelated eager work of the same context and of torch between the replays
        ctx.gram_exact(arr, other, X.FP32C)
        torch.ones(256, 256, device=dev).sum().item()
        torch.cuda.synchronize()
        g.launch(s)
        s.synchronize()
        got = [tuple(outs[i]) for i in range(len(forms))] + [gram]
        for w, o in zip(want[:-1], got[:-1]):
            for a, c in zip(w, o):
                assert torch.equal(a, c), r
        assert torch.equal(want[-1], got[-1]), r
    # networks and contexts are not destroyed under a live graph
    assert X._lib.xlmimo_mlp_destroy(mlp.h) == X.EINVAL
    g.close()
    mlp.close()


def test_graph_capture_refuses_cold_and_foreign_calls(X, ctx):
    arr, drops, b, rho = _sweep_setup(X)
    s = torch.cuda.Stream()
    ctx.gram_exact(arr, b, X.FP32H, stream=s)  # warm this shape only
    s.synchronize()
    cold = X.Batch(W.polar_drops(W.rng_for(9), 17, 5, 2000, (5.0, 50.0), (-60.0, 60.0)))
    out = torch.empty(2 * cold.gram_elems, dtype=torch.float64, device=b.pos.device)
    out_b = torch.empty(2 * b.gram_elems, dtype=torch.float64, device=b.pos.device)
    ctx.graph_begin(s)
    with pytest.raises(X.XlmimoError, match="launch plan during graph capture"):
        ctx.gram_exact(arr, cold, X.FP32H, out=out, stream=s)
    with pytest.raises(X.XlmimoError, match="capturing stream"):
        ctx.gram_exact(arr, b, X.FP32H, out=out_b)
    with pytest.raises(X.XlmimoError, match="capture failed"):
        ctx.graph_end(s)
    # the context and the stream work normally afterwards
    g1 = ctx.gram_exact(arr, cold, X.FP32H, stream=s)
    s.synchronize()
    g2 = ctx.gram_exact(arr, cold, X.FP32H)
    torch.cuda.synchronize()
    assert torch.equal(g1, g2)


def test_autotune_keeps_parity_and_determinism(X, ctx):
    ns = [3000, 70001, 12345, 257, 40000, 131072]
    ks = [16, 5, 33, 2, 16, 9]
    rng = np.random.default_rng(31)
    pos = []
    for k in ks:
        r = rng.uniform(2.0, 40.0, k)
        t = np.deg2rad(rng.uniform(-70.0, 70.0, k))
        pos.append(np.stack([r * np.cos(t), r * np.sin(t), np.zeros(k)], axis=-1))
    drops = W._pack(ns, ks, np.concatenate(pos))
    arr = W.ula(1, W.LAMBDA_28GHZ)
    b = X.Batch(drops)
    for prec in (X.FP32H, X.FP32C):
        res = ctx.autotune_exact(arr, b, prec)
        assert res["chunk"] % 128 == 0 and 1024 <= res["chunk"] <= 131072
        assert res["grid"] >= 1 and res["ms"] > 0
        g1 = ctx.gram_exact(arr, b, prec).clone()
        g2 = ctx.gram_exact(arr, b, prec)
        torch.cuda.synchronize()
        assert torch.equal(g1, g2)
        g = b.split(g1)
        for d in range(drops.n_drops):
            ref = och.gram_exact(arr.with_n(ns[d]), drops.users_of(d))
            assert och.normwise_error(g[d], ref) < 1e-5, (prec, d)


def test_autotune_sweep_points(X, ctx):
    arr, drops, b, rho = _sweep_setup(X)
    n_list = [256, 1024, 4096]
    e0, _, _ = ctx.capacity_sweep(arr, n_list, b, X.FORM_EXACT_FP32H, rho, X.ZF | X.MMSE)
    e0 = e0.clone()
    for n in n_list:
        res = ctx.autotune_exact(arr, b, X.FP32H, n_elems=n)
        assert res["chunk"] % 128 == 0
    e1, _, _ = ctx.capacity_sweep(arr, n_list, b, X.FORM_EXACT_FP32H, rho, X.ZF | X.MMSE)
    torch.cuda.synchronize()
    assert torch.allclose(e0, e1, rtol=1e-6, atol=0)
    with pytest.raises(X.XlmimoError, match="n_elems"):
        ctx.autotune_exact(W.ArraySpec(W.GEOM_UPA, 8, 8, 0.0015, 0.003), b, X.FP32H, n_elems=64)
