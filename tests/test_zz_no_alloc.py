"""The allocation-free exact Gram (xlmimo_gram_exact_noalloc) against the
context's exact Gram (xlmimo_gram_exact) and the FP64 oracle, through the C ABI.

Both entry points run the same kernels; with the same work-item partition
(an untuned context) their Grams are bit-identical.  Where the allocation-free
path must lengthen its work items to fit its static scratch, only the FP32
summation order differs, and the two agree to the exact form's tolerance
(1e-5 normwise).  Every call on a GPU shares one static array, so two calls in
a row, the second with a smaller batch, must each match on their own."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import channel as och

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
    c = X.Context(0)   # a context of its own: no autotuned shapes
    yield c
    c.close()


def _drops(ns, ks, seed):
    rng = np.random.default_rng(seed)
    pos = []
    for k in ks:
        r = rng.uniform(2.0, 40.0, k)
        t = np.deg2rad(rng.uniform(-70.0, 70.0, k))
        pos.append(np.stack([r * np.cos(t), r * np.sin(t), np.zeros(k)], axis=-1))
    return W._pack(ns, ks, np.concatenate(pos))


def _oracle_check(arr, drops, b, out, precision, picks):
    g = b.split(out)
    for d in picks:
        ref = och.gram_exact(arr.with_n(int(drops.n_elems[d])), drops.users_of(d))
        err = och.normwise_error(g[d], ref)
        assert err < TOL[precision], (precision, d, int(drops.n_elems[d]), int(drops.n_users[d]), err)


def _run_pair(X, ctx, arr, drops, precision):
    b = X.Batch(drops)
    p = getattr(X, precision)
    print(f"no-alloc exact Gram: {precision}, {drops.n_drops} drops, N <= {int(drops.n_elems.max())}, "
          f"K <= {int(drops.n_users.max())}", flush=True)
    out_na = torch.full((2 * b.gram_elems,), float("nan"), dtype=torch.float64, device=b.pos.device)
    ctx.gram_exact_noalloc(arr, b, p, out_na)
    out_ref = ctx.gram_exact(arr, b, p)
    torch.cuda.synchronize()
    return b, out_na, out_ref


@pytest.mark.parametrize("precision", ["FP32H", "FP64", "FP32C"])
def test_two_calls_in_a_row_match_the_context_path(X, ctx, precision):
    arr = W.ula(1, W.LAMBDA_28GHZ)
    # first call: ragged N (1 .. 70001) and K across the 16-user blocks (1 .. 64)
    ns1 = [1, 2, 3, 17, 255, 1000, 4097, 70001, 300, 5000, 4096, 12345, 65536, 2048]
    ks1 = [1, 2, 15, 16, 17, 32, 33, 64, 4, 5, 16, 7, 16, 64]
    d1 = _drops(ns1, ks1, seed=71)
    b1, na1, ref1 = _run_pair(X, ctx, arr, d1, precision)
    assert torch.equal(na1, ref1), "first call: not bit-identical to xlmimo_gram_exact"
    _oracle_check(arr, d1, b1, na1, precision, picks=[0, 3, 6, 7, 11, 13])
    keep = na1.clone()
    # second call, smaller: fewer drops, fewer users, shorter arrays
    ns2 = [3, 129, 1024, 777]
    ks2 = [2, 9, 16, 1]
    d2 = _drops(ns2, ks2, seed=72)
    b2, na2, ref2 = _run_pair(X, ctx, arr, d2, precision)
    assert torch.equal(na2, ref2), "second call: not bit-identical to xlmimo_gram_exact"
    _oracle_check(arr, d2, b2, na2, precision, picks=range(d2.n_drops))
    assert torch.equal(na1, keep), "the first call's output changed"


def test_uneven_batch_and_the_sweep_shape(X, ctx):
    # the uneven-batch law (N ~ U{1024..262144}, K ~ U{2..32}), then a sweep point
    arr, drops, _ = W.uneven(n_drops=256)
    b, na, ref = _run_pair(X, ctx, arr, drops, "FP32H")
    assert torch.equal(na, ref)
    _oracle_check(arr, drops, b, na, "FP32H", picks=[0, 1, 255])
    arr2, d2, _ = W.sweep(n_drops=2000, n_list=(16384,))
    b2, na2, ref2 = _run_pair(X, ctx, arr2, d2, "FP32H")
    assert torch.equal(na2, ref2)
    _oracle_check(arr2, d2, b2, na2, "FP32H", picks=[0, 1999])


def test_lengthened_items_agree_to_tolerance(X, ctx):
    # 1000 drops of 64 users at N = 65536: the context's default partition needs
    # more partial sums than the static scratch holds, so the allocation-free
    # path runs one item per drop (FP32 sums in another order)
    ns = [65536] * 1000
    ks = [64] * 1000
    d = _drops(ns, ks, seed=73)
    arr = W.ula(1, W.LAMBDA_28GHZ)
    b, na, ref = _run_pair(X, ctx, arr, d, "FP32C")
    g_na, g_ref = b.split(na), b.split(ref)
    worst = max(och.normwise_error(g_na[i], g_ref[i]) for i in range(0, 1000, 37))
    assert worst < 1e-5, worst
    _oracle_check(arr, d, b, na, "FP32C", picks=[0, 999])


def test_limits_are_rejected_on_the_host(X, ctx):
    arr = W.ula(1, W.LAMBDA_28GHZ)
    # K above XLMIMO_MAX_USERS
    d = _drops([1024], [65], seed=74)
    b = X.Batch(d)
    out = torch.empty(2 * b.gram_elems, dtype=torch.float64, device=b.pos.device)
    with pytest.raises(X.XlmimoError, match="K = 65"):
        ctx.gram_exact_noalloc(arr, b, X.FP32H, out)
    # more partial sums than the static array holds even at one item per drop
    # (1300 drops x 64 users: 1300 x 53 KB > 64 MiB)
    d = _drops([1024] * 1300, [64] * 1300, seed=75)
    b = X.Batch(d)
    out = torch.empty(2 * b.gram_elems, dtype=torch.float64, device=b.pos.device)
    with pytest.raises(X.XlmimoError, match="scratch"):
        ctx.gram_exact_noalloc(arr, b, X.FP32H, out)
    # an empty batch is a no-op
    e = W._pack([], [], np.zeros((0, 3)))
    ctx.gram_exact_noalloc(arr, X.Batch(e), X.FP32H, out)
    torch.cuda.synchronize()
