"""The allocation-free filter entry point against chebfd_filter_apply.

Both run the same kernels in the same order, so the filtered block and the
Chebyshev moments must agree bit for bit.  Two calls in a row, the second
with a smaller input (fewer partial-sum rows than the first left in the
shared device array), on SELL and on the matrix-free stencil; and a call
whose partial sums exceed the fixed array is rejected before any launch.
"""
import numpy as np
import pytest

import chebfd_inputs as inp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1510_04895_amd import binding as B
    assert torch.cuda.is_available()
    return torch, B, B.Context(0)


def _run(torch, B, ctx, H, fn, X0, gam, a, b, dtype):
    X = torch.from_numpy(X0).to(dtype).cuda()
    U, W = torch.empty_like(X), torch.empty_like(X)
    n_s = X.shape[1]
    mom = torch.full((2 * (len(gam) - 1) + 1, n_s), float("nan"), dtype=torch.float64,
                     device="cuda")
    fn(ctx, H, gam, a, b, X, U, W, moments=mom)
    torch.cuda.synchronize()
    return X.cpu().numpy(), mom.cpu().numpy()


@pytest.mark.parametrize("storage", ["sell", "stencil"])
@pytest.mark.parametrize("dtype_name", ["complex128", "complex64"])
def test_noalloc_matches_filter_apply(env, storage, dtype_name):
    torch, B, ctx = env
    dtype = getattr(torch, dtype_name)
    st = B.STORAGE_SELL if storage == "sell" else B.STORAGE_STENCIL
    # first a larger problem, then a smaller one (the second call's partial
    # rows are a prefix of what the first left in the shared array)
    for L, n_s, n_p, seed in (((16, 16, 8), 24, 40, 3), ((6, 4, 5), 6, 17, 4)):
        print(f"noalloc case storage={storage} dtype={dtype_name} L={L} n_s={n_s} n_p={n_p}",
              flush=True)
        H = B.Matrix.ti(ctx, L, pbc=3, V=1.0, seed=seed, storage=st)
        info = H.info()
        a, b = info["g_lo"], info["g_hi"]
        X0 = inp.random_block(info["n"], n_s, seed=seed + 10)
        gam = inp.random_gamma(n_p, seed=seed + 20)
        Xr, mr = _run(torch, B, ctx, H, B.chebfd_filter_apply, X0, gam, a, b, dtype)
        Xn, mn = _run(torch, B, ctx, H, B.chebfd_filter_apply_noalloc, X0, gam, a, b, dtype)
        assert np.isfinite(mr).all() and np.isfinite(Xr).all()
        assert np.array_equal(Xn, Xr)
        assert np.array_equal(mn, mr)
        # and without moments
        Xm = torch.from_numpy(X0).to(dtype).cuda()
        U, W = torch.empty_like(Xm), torch.empty_like(Xm)
        B.chebfd_filter_apply_noalloc(ctx, H, gam, a, b, Xm, U, W)
        torch.cuda.synchronize()
        assert np.array_equal(Xm.cpu().numpy(), Xr)
        H.close()


def test_noalloc_rejects_oversized_partials(env):
    """32x32x32 SELL-32 (one row per slot) with 256 columns needs 16384 row
    blocks x 256 x 24 B = 100.7 MB of partial sums, more than the 64 MiB
    array."""
    torch, B, ctx = env
    B.chebfd_set_tuning(ctx, "row_group", 1)
    try:
        H = B.Matrix.ti(ctx, (32, 32, 32), pbc=3, V=1.0, seed=1)
    finally:
        B.chebfd_set_tuning(ctx, "row_group", -1)
    n = H.info()["n"]
    X = torch.zeros((n, 256), dtype=torch.complex128, device="cuda")
    U, W = torch.empty_like(X), torch.empty_like(X)
    mom = torch.zeros((2 * 8 + 1, 256), dtype=torch.float64, device="cuda")
    gam = inp.random_gamma(8, seed=1)
    with pytest.raises(B.ChebFDError) as e:
        B.chebfd_filter_apply_noalloc(ctx, H, gam, -9.0, 9.0, X, U, W, moments=mom)
    assert e.value.code == -1 and "64" in str(e.value)
    H.close()
