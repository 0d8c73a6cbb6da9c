"""Learned correction on the GPU against the FP64 MLP reference.

Forward outputs and gradients are compared with the oracle evaluated at the
same BF16-rounded weights and inputs; the GPU also rounds every activation and
back-propagated gradient to BF16 between layers, so the tolerance is a
relative Frobenius error of 2e-2 per parameter tensor (5e-2 for the first
layer's weights, whose inputs are six BF16 features).
"""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import channel as och
from oracle import closedform as ocf
from oracle import mlp as OM

pytestmark = pytest.mark.gpu

WIDTH, DEPTH = 256, 4


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


def bf16_round(a):
    """Round float64 values to the nearest bfloat16 (ties to even)."""
    f = np.asarray(a, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _pairs(X, ctx, mlp, n_drops=6, k=7, stream=9):
    arr, drops = W.learned_drops(n_drops, stream=stream, k=k)
    b = X.Batch(drops)
    gcf, _ = ctx.gram_closedform(arr, b, X.CF_GATED)
    gex = ctx.gram_exact(arr, b, X.FP64)
    return arr, drops, mlp.pair_inputs(arr, b, gcf, gex), gcf, gex, b


def test_pair_inputs_match_oracle(X, ctx):
    mlp = X.MLP(ctx, WIDTH, DEPTH)
    arr, drops, pi, gcf, gex, b = _pairs(X, ctx, mlp)
    torch.cuda.synchronize()
    feat = pi.feat.float().cpu().numpy()
    aux = pi.aux.cpu().numpy()
    tgt = pi.target.cpu().numpy()
    pm = pi.pmap.cpu().numpy()
    p = 0
    for d in range(drops.n_drops):
        u = drops.users_of(d)
        n = int(drops.n_elems[d])
        a = arr.with_n(n)
        g_ex = och.gram_exact(a, u)
        g_cf = ocf.gram_closedform(a, u, n, ocf.VARIANT_GATED)
        k = len(u)
        for i in range(k):
            for j in range(i + 1, k):
                sc = math.sqrt(g_cf[i, i].real * g_cf[j, j].real)
                f, ph = OM.pair_inputs(u[i, 0], u[i, 1], u[j, 0], u[j, 1], n, a.spacing, a.wavelength, sc)
                assert np.allclose(feat[p, :6], bf16_round(f), rtol=0, atol=1e-12)
                assert np.all(feat[p, 6:] == 0)
                got = aux[p, 0:6:2] + 1j * aux[p, 1:6:2]
                assert np.all(np.abs(got - ph) <= 2e-6 * np.maximum(np.abs(ph), 1.0)), (got, ph)
                assert aux[p, 6] == pytest.approx(sc, rel=1e-6)
                want = g_ex[i, j] / math.sqrt(g_ex[i, i].real * g_ex[j, j].real) \
                    - g_cf[i, j] / math.sqrt(g_cf[i, i].real * g_cf[j, j].real)
                assert abs(tgt[p, 0] + 1j * tgt[p, 1] - want) < 1e-6
                assert pm[p, 0] == d and pm[p, 1] == 64 * i + j
                p += 1
    assert p == pi.n
    mlp.close()


def test_forward_and_gradients_match_oracle(X, ctx):
    rng = np.random.default_rng(11)
    mlp = X.MLP(ctx, WIDTH, DEPTH)
    params = OM.init_params(rng, WIDTH, DEPTH)
    params[-OM.N_OUT:] = rng.normal(size=OM.N_OUT) * 0.1
    params[-1] = -4.0
    mlp.set_params(params.astype(np.float32))
    assert np.array_equal(mlp.get_params(), params.astype(np.float32))
    arr, drops, pi, *_ = _pairs(X, ctx, mlp, n_drops=40, k=16, stream=12)   # 4800 pairs: several tiles, ragged
    out = mlp.forward(pi)
    loss, grad = mlp.loss_grad(pi)
    torch.cuda.synchronize()
    pb = bf16_round(params)
    # biases stay FP32 on the GPU
    for (o, i), off in zip(OM.layer_shapes(WIDTH, DEPTH), np.cumsum([0] + [o * i + o for o, i in OM.layer_shapes(WIDTH, DEPTH)])):
        pb[off + o * i: off + o * i + o] = params[off + o * i: off + o * i + o].astype(np.float32)
    x = pi.feat.float().cpu().numpy()[:, :6].astype(np.float64)
    ph = (pi.aux[:, 0:6:2] + 1j * pi.aux[:, 1:6:2]).cpu().numpy().astype(np.complex128)
    tg = (pi.target[:, 0] + 1j * pi.target[:, 1]).cpu().numpy().astype(np.complex128)
    ref_out, _ = OM.forward(pb, x, WIDTH, DEPTH)
    o = out.cpu().numpy()
    assert np.linalg.norm(o - ref_out) / np.linalg.norm(ref_out) < 2e-2
    ref_loss, ref_g = OM.loss_grad(pb, x, ph, tg, WIDTH, DEPTH)
    assert loss.item() == pytest.approx(ref_loss, rel=1e-2)
    g = grad.cpu().numpy()
    off = 0
    for li, (o_, i_) in enumerate(OM.layer_shapes(WIDTH, DEPTH)):
        for name, size in (("W", o_ * i_), ("b", o_)):
            a, r = g[off:off + size], ref_g[off:off + size]
            err = np.linalg.norm(a - r) / np.linalg.norm(r)
            tol = 5e-2 if (li == 0 and name == "W") else 2e-2
            assert err < tol, (li, name, err)
            off += size


def test_training_reduces_loss_and_adam_matches(X, ctx):
    rng = np.random.default_rng(13)
    mlp = X.MLP(ctx, 64, 2)
    params = OM.init_params(rng, 64, 2).astype(np.float32)
    mlp.set_params(params)
    arr, drops, pi, *_ = _pairs(X, ctx, mlp, n_drops=60, k=16, stream=14)
    # one Adam step equals the reference update at the same gradient: first step moves by ~lr * sign(g)
    loss, grad = mlp.loss_grad(pi)
    mlp.train_step(pi, 1e-3)
    torch.cuda.synchronize()
    g = grad.cpu().numpy().astype(np.float64)
    opt = OM.Adam(params.size, lr=1e-3)
    want = opt.step(params.astype(np.float64), g)
    got = mlp.get_params()
    assert np.allclose(got, want, rtol=0, atol=2e-6)
    losses = []
    for s in range(300):
        l = mlp.train_step(pi, 2e-3)
        if s % 50 == 0:
            losses.append(l.item())
    assert losses[-1] < losses[0] - 1.0, losses


def test_multi_step_training_equals_single_steps(X, ctx):
    # xlmimo_mlp_train enqueues the same kernels as repeated xlmimo_mlp_train_step calls on
    # consecutive batch slices (wrapping around): bit-identical parameters and losses
    rng = np.random.default_rng(15)
    params = OM.init_params(rng, 256, 4).astype(np.float32)
    arr, drops, pi, *_ = _pairs(X, ctx, X.MLP(ctx, 256, 4), n_drops=40, k=16, stream=16)   # 4800 pairs
    batch, steps = 1000, 11
    lr = np.linspace(3e-3, 1e-4, steps).astype(np.float32)
    a, b = X.MLP(ctx, 256, 4), X.MLP(ctx, 256, 4)
    a.set_params(params)
    b.set_params(params)
    la = []
    nb = pi.n // batch
    for s_ in range(steps):
        o = (s_ % nb) * batch
        la.append(a.train_step(pi.slice(o, o + batch), float(lr[s_])).item())
    lb = torch.empty(steps, dtype=torch.float64, device=pi.aux.device)
    b.train(pi, batch, lr, lb)
    torch.cuda.synchronize()
    assert np.array_equal(a.get_params(), b.get_params())
    assert np.array_equal(np.array(la), lb.cpu().numpy())


@pytest.mark.parametrize("width,depth", [(512, 9), (256, 4), (128, 4), (64, 4)])
def test_gradient_paths_agree(X, ctx, width, depth):
    # Two implementations of each training pass, on one batch of 16384 pairs and on its 32
    # sub-batches of 512.  Width 512 runs the layer GEMMs: a network whose split-K weight-gradient
    # slices fit the library's budget runs the grouped weight-gradient launch on a transposed weight
    # copy (every sub-batch here); one whose slices do not (2.1 M parameters x 32 slices at 16384
    # pairs) reduces each layer right after its GEMM.  Widths 256, 128 and 64 run the fused forward and
    # input-gradient passes (at width 256 with 64-pair tiles at 16384 pairs and 32-pair tiles below).  The
    # gradient of the mean loss over 16384 pairs is the mean of the 32 sub-batch gradients: the 1/n
    # scalings are powers of two, so every BF16 rounding scales exactly and only the FP32 summation
    # orders differ.
    rng = np.random.default_rng(37)
    mlp = X.MLP(ctx, width, depth)
    params = OM.init_params(rng, width, depth)
    params[-OM.N_OUT:] = rng.normal(size=OM.N_OUT) * 0.1
    mlp.set_params(params.astype(np.float32))
    arr, drops, pi, *_ = _pairs(X, ctx, mlp, n_drops=137, k=16, stream=37)   # 16440 pairs
    n, sub = 16384, 512
    loss_full, grad_full = mlp.loss_grad(pi.slice(0, n))
    grads, losses = [], []
    for a in range(0, n, sub):
        l_, g_ = mlp.loss_grad(pi.slice(a, a + sub))
        grads.append(g_.double().cpu().numpy())
        losses.append(l_.item())
    g_mean = np.mean(grads, axis=0)
    g_full = grad_full.double().cpu().numpy()
    assert abs(loss_full.item() - np.mean(losses)) <= 1e-9 * abs(loss_full.item())
    off = 0
    for li, (o, i) in enumerate(OM.layer_shapes(width, depth)):
        for name, m in (("W", o * i), ("b", o)):
            a_, b_ = g_full[off:off + m], g_mean[off:off + m]
            err = np.linalg.norm(a_ - b_) / max(np.linalg.norm(b_), 1e-30)
            assert err < 1e-5, (li, name, err)
            off += m
    mlp.close()


@pytest.mark.parametrize("width,depth,n_drops", [(64, 2, 3), (128, 3, 5), (256, 1, 2)])
def test_fused_forward_other_shapes(X, ctx, width, depth, n_drops):
    # the fused inference kernel at every width it supports, with a ragged last tile
    rng = np.random.default_rng(width + depth)
    mlp = X.MLP(ctx, width, depth)
    params = OM.init_params(rng, width, depth)
    params[-OM.N_OUT:] = rng.normal(size=OM.N_OUT) * 0.1
    mlp.set_params(params.astype(np.float32))
    arr, drops, pi, *_ = _pairs(X, ctx, mlp, n_drops=n_drops, k=11, stream=20 + width)   # 55 pairs per drop
    out = mlp.forward(pi).cpu().numpy()
    pb = bf16_round(params)
    shapes = OM.layer_shapes(width, depth)
    off = 0
    for o, i in shapes:
        pb[off + o * i: off + o * i + o] = params[off + o * i: off + o * i + o].astype(np.float32)
        off += o * i + o
    x = pi.feat.float().cpu().numpy()[:, :6].astype(np.float64)
    ref, _ = OM.forward(pb, x, width, depth)
    assert np.linalg.norm(out - ref) / np.linalg.norm(ref) < 2e-2
    mlp.close()


@pytest.mark.parametrize("width,depth", [(256, 4), (128, 3), (64, 2)])
def test_fused_forward_at_kernel_precision(X, ctx, width, depth):
    # The fused forward against the oracle's network evaluated at the kernel's precision:
    # BF16 weights and inputs, FP32 biases, FP64 sums, each hidden activation rounded to
    # BF16 after the GELU.  What is left is the FP32 accumulation and the rare BF16
    # rounding it flips, so an error in the activation (its polynomial, clamp or max)
    # at the 1e-3 level fails here, where the plain FP64 comparison allows 2e-2.
    rng = np.random.default_rng(29 + width)
    mlp = X.MLP(ctx, width, depth)
    params = OM.init_params(rng, width, depth)
    mlp.set_params(params.astype(np.float32))
    arr, drops, pi, *_ = _pairs(X, ctx, mlp, n_drops=20, k=16, stream=31 + width)   # 2400 pairs, ragged tile
    out = mlp.forward(pi).cpu().numpy().astype(np.float64)
    layers = OM.unpack(params, width, depth)
    a = pi.feat.float().cpu().numpy()[:, :6].astype(np.float64)
    for li, (w, b) in enumerate(layers):
        z = a @ bf16_round(w).T + np.asarray(b, np.float32).astype(np.float64)
        a = bf16_round(OM.gelu(z)) if li + 1 < len(layers) else z
    err = np.linalg.norm(out - a) / np.linalg.norm(a)
    print(f"fused forward, width {width}, depth {depth}: {err:.2e} against the BF16-activation network")
    assert err < 1e-3, (width, depth, err)
    mlp.close()


def test_fallback_recomputes_flagged_drops_exactly(X, ctx):
    # Drops where the predicted log-variance exceeds log_var_max for some pair are recomputed by the
    # exact FP32H kernel over their own work items only (selected on the device); the other drops keep
    # the corrected closed form.  The threshold splits the drops about in half.
    rng = np.random.default_rng(21)
    mlp = X.MLP(ctx, 64, 2)
    mlp.set_params(OM.init_params(rng, 64, 2).astype(np.float32))
    arr, drops = W.learned_drops(24, stream=31, k=9)
    b = X.Batch(drops)
    gcf, _ = ctx.gram_closedform(arr, b, X.CF_GATED_QUAD)
    pi = mlp.pair_inputs(arr, b, gcf)
    s = mlp.forward(pi)[:, 6].cpu().numpy()
    pm = pi.pmap.cpu().numpy()
    smax = np.full(drops.n_drops, -np.inf, np.float32)
    np.maximum.at(smax, pm[:, 0], s)
    order = np.sort(smax)
    thr = float(0.5 * (order[11] + order[12]))
    assert order[11] < thr < order[12]
    out, st = ctx.gram_closedform_mlp(arr, b, mlp, X.CF_GATED_QUAD, thr)
    kept, st_kept = ctx.gram_closedform_mlp(arr, b, mlp, X.CF_GATED_QUAD, 1e30)
    ex = ctx.gram_exact(arr, b, X.FP32H)
    torch.cuda.synchronize()
    fell = (st.cpu().numpy() & X.ST_FELL_BACK) != 0
    assert np.array_equal(fell, smax > thr) and fell.sum() == 12
    assert not np.any(st_kept.cpu().numpy() & X.ST_FELL_BACK)
    g, gk, ge = b.split(out), b.split(kept), b.split(ex)
    for d in range(drops.n_drops):
        assert np.array_equal(g[d], ge[d] if fell[d] else gk[d]), d
    mlp.close()
