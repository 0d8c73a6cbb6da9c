"""The FP32H exact Gram's channel paths against the FP64 oracle.

Items whose users are all at least 368 element spacings from the array line
(plane) evaluate each lane's run of 16 consecutive elements from an FP64 distance
and phase at the run's centre plus FP32 expansions of the phase and amplitude
along the run; in batches of at most 32 users, items whose users are all at least
184 spacings away take a second tier of the expansion (two more phase terms, one
more amplitude term); other items evaluate every element in FP64.  Each case below
is built so that one path must run (users all far, one user between 184 and 368
spacings, or one user nearer), for the ULA and the UPA, both amplitude models and
three spacings, and each is held to the exact form's tolerance (1e-5 normwise)
against the oracle, with ragged element counts so that the last run of an item is
partial."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import channel as och

pytestmark = pytest.mark.gpu

TOL = 1e-5
XMIN = 368.0   # element spacings
XMIN2 = 184.0  # the second expansion tier


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


def _users(rng, k, x_lo, x_hi, y_span, z_span=0.0):
    x = rng.uniform(x_lo, x_hi, k)
    y = rng.uniform(-y_span, y_span, k)
    z = rng.uniform(-z_span, z_span, k) if z_span else np.zeros(k)
    return np.stack([x, y, z], axis=-1)


def _check(X, ctx, arr, drops, what):
    b = X.Batch(drops)
    print(f"{what}: {drops.n_drops} drops, N up to {int(drops.n_elems.max())}", flush=True)
    g = b.split(ctx.gram_exact(arr, b, X.FP32H))
    torch.cuda.synchronize()
    worst = 0.0
    for d in range(drops.n_drops):
        a = arr.with_n(int(drops.n_elems[d])) if arr.geometry == W.GEOM_ULA else arr
        ref = och.gram_exact(a, drops.users_of(d))
        err = och.normwise_error(g[d], ref)
        worst = max(worst, err)
        assert err < TOL, (what, d, err)
        assert np.array_equal(g[d], g[d].conj().T)
    return worst


@pytest.mark.parametrize("amp", [W.AMP_FREESPACE, W.AMP_PNUSW])
@pytest.mark.parametrize("spacing_lam", [0.5, 1.0, 0.25])
def test_ula_far_and_near_users(X, ctx, amp, spacing_lam):
    lam = W.LAMBDA_28GHZ
    d = spacing_lam * lam
    x_far = XMIN * d * 1.001
    rng = np.random.default_rng(int(spacing_lam * 100) + amp)
    ns = [1000, 4099, 70001, 129, 16384]
    ks = [16, 9, 16, 32, 5]
    far = [_users(rng, k, x_far, x_far + 40.0, 30.0) for k in ks]          # expansion path
    mid = [u.copy() for u in far]
    for u in mid:
        u[-1, 0] = XMIN2 * d * 1.001                                         # one user at 184 d: second tier
    near = [u.copy() for u in far]
    for u in near:
        u[-1, 0] = XMIN2 * d * 0.8                                           # one user nearer: FP64 path
    arr = W.ula(1, lam, amp, spacing=d)
    w_far = _check(X, ctx, arr, W._pack(ns, ks, np.concatenate(far)), "far users")
    w_mid = _check(X, ctx, arr, W._pack(ns, ks, np.concatenate(mid)), "one user at 184 spacings")
    w_near = _check(X, ctx, arr, W._pack(ns, ks, np.concatenate(near)), "one near user")
    print(f"worst normwise error: far {w_far:.2e}, 184 d {w_mid:.2e}, near {w_near:.2e}", flush=True)


@pytest.mark.parametrize("amp", [W.AMP_FREESPACE, W.AMP_PNUSW])
def test_upa_second_tier(X, ctx, amp):
    # users between 184 and 368 spacings of a panel whose columns hold whole runs: the second tier
    lam = W.LAMBDA_100GHZ_UPA
    d = lam / 2
    rng = np.random.default_rng(184 + amp)
    k = 16
    users = [_users(rng, k, XMIN2 * d * 1.001, XMIN * d * 0.99, 0.3, 0.3) for _ in range(3)]
    arr = W.ArraySpec(W.GEOM_UPA, 48, 32, d, lam, amp)
    drops = W._pack([48 * 32] * 3, [k] * 3, np.concatenate(users))
    w = _check(X, ctx, arr, drops, "UPA 48x32, users at 184-368 spacings")
    print(f"worst normwise error {w:.2e}", flush=True)


@pytest.mark.parametrize("ny,nz", [(40, 64), (33, 24), (16, 21)])
def test_upa_runs_along_columns(X, ctx, ny, nz):
    # n_z a multiple of 16: every run of 16 elements stays in one column (expansion path);
    # otherwise the per-element FP64 distance
    lam = W.LAMBDA_100GHZ_UPA
    d = lam / 2
    rng = np.random.default_rng(ny * 100 + nz)
    k = 12
    users = [_users(rng, k, XMIN * d * 1.01, 20.0, 5.0, 5.0) for _ in range(3)]
    arr = W.ArraySpec(W.GEOM_UPA, ny, nz, d, lam, W.AMP_FREESPACE)
    drops = W._pack([ny * nz] * 3, [k] * 3, np.concatenate(users))
    _check(X, ctx, arr, drops, f"UPA {ny}x{nz}")


def test_sweep_drops_at_the_largest_aperture(X, ctx):
    # the sweep's user law (x >= 2.5 m, far above 368 d = 1.97 m) at N = 262144
    arr, drops, _ = W.sweep(n_drops=6, n_list=(262144,))
    w = _check(X, ctx, arr, drops, "sweep drops, N = 262144")
    print(f"worst normwise error {w:.2e}", flush=True)


@pytest.mark.parametrize("amp", [W.AMP_FREESPACE, W.AMP_PNUSW])
def test_64_user_drops(X, ctx, amp):
    # Drops of 49-64 users (four 16-user blocks) run the block-per-wave kernel: each wave evaluates
    # one block and the products are shared out through LDS.  A batch of such drops alone (no
    # 33-48-user drop) takes the kernel without FP32C paths; far users (expansion) and one near
    # user (per-element distance), ragged N.
    lam = W.LAMBDA_28GHZ
    d = 0.5 * lam
    x_far = XMIN * d * 1.001
    rng = np.random.default_rng(64 + amp)
    ns = [4099, 1000, 20000]
    ks = [64, 49, 64]
    far = [_users(rng, k, x_far, x_far + 30.0, 20.0) for k in ks]
    near = [u.copy() for u in far]
    for u in near:
        u[5, 0] = x_far * 0.4
    arr = W.ula(1, lam, amp)
    w_far = _check(X, ctx, arr, W._pack(ns, ks, np.concatenate(far)), "64 users, far")
    w_near = _check(X, ctx, arr, W._pack(ns, ks, np.concatenate(near)), "64 users, one near")
    # beside 16- and 33-user drops: the general kernel, whose 4-block drops take the same path
    mixed = W._pack(ns + [777, 3000], ks + [16, 33],
                    np.concatenate(far + [_users(rng, 16, x_far, x_far + 30.0, 20.0),
                                          _users(rng, 33, x_far, x_far + 30.0, 20.0)]))
    w_mixed = _check(X, ctx, arr, mixed, "64 users beside 16 and 33")
    print(f"worst normwise error: far {w_far:.2e}, near {w_near:.2e}, mixed {w_mixed:.2e}", flush=True)


@pytest.mark.parametrize("ny,nz", [(24, 32), (20, 40)])
def test_upa_64_users(X, ctx, ny, nz):
    # the block-per-wave kernel on a UPA: runs of 16 along the columns (n_z = 32) or the
    # per-element distance (n_z = 40)
    lam = W.LAMBDA_100GHZ_UPA
    d = lam / 2
    rng = np.random.default_rng(ny * 1000 + nz)
    k = 64
    users = [_users(rng, k, XMIN * d * 1.01, 3.0, 1.5, 1.5) for _ in range(2)]
    arr = W.ArraySpec(W.GEOM_UPA, ny, nz, d, lam, W.AMP_FREESPACE)
    drops = W._pack([ny * nz] * 2, [k] * 2, np.concatenate(users))
    _check(X, ctx, arr, drops, f"UPA {ny}x{nz}, K = 64")
