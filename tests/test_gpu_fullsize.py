"""Parity at the full 64x64x32 size (N = 524,288, 256 search vectors) in the
launch configuration the benchmark times: the fused filter against the CPU
reference on the whole block, and the complete solve checked through
properties the reference recomputes at any size (residuals from its own
sparse product, orthonormality, count and Kramers degeneracy)."""
import math

import numpy as np
import pytest

import chebfd_inputs as inp

pytestmark = pytest.mark.gpu

W = inp.WORKLOADS["ti_64x64x32"]


@pytest.fixture(scope="module")
def env(orc):
    import torch
    from paper_1510_04895_amd import binding as B
    assert torch.cuda.is_available()
    ctx = B.Context(0)
    Hr = orc.ti_hamiltonian(*W["L"], pbc=W["pbc"], V=W["V"], seed=W["seeds"][0])
    return torch, B, ctx, Hr


def _matrix(B, ctx, storage):
    return B.Matrix.ti(ctx, W["L"], pbc=W["pbc"], V=W["V"], seed=W["seeds"][0],
                       storage=B.STORAGE_SELL if storage == "sell" else B.STORAGE_STENCIL,
                       sell_C=W["sell_C"], sell_sigma=W["sell_sigma"])


@pytest.mark.parametrize("storage", ["sell", "stencil"])
@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_fused_filter_full_size(env, orc, storage, prec):
    torch, B, ctx, Hr = env
    a, b = orc.gershgorin(Hr)
    n_s, n_p = W["n_s"], 12
    X = inp.random_block(Hr.n, n_s, seed=21)
    if prec == "c64":
        X = X.astype(np.complex64).astype(np.complex128)
    gam = orc.gamma(-W["delta"], W["delta"], a, b, n_p)
    ref = orc.filter_block(Hr, a, b, gam, X)
    H = _matrix(B, ctx, storage)
    dt = torch.complex128 if prec == "c128" else torch.complex64
    Xd = torch.from_numpy(X).to(dt).cuda()
    Ud, Wd = torch.empty_like(Xd), torch.empty_like(Xd)
    B.chebfd_filter_apply(ctx, H, gam, a, b, Xd, Ud, Wd)
    torch.cuda.synchronize()
    got = Xd.cpu().numpy().astype(np.complex128)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    el = np.abs(got - ref).max() / np.abs(ref).max()
    tol = 1e-12 * n_p if prec == "c128" else 30 * math.sqrt(n_p) * 2.0 ** -24
    assert err < tol and el < tol, (err, el)


def _oracle_window():
    """Eigenvalues of the 64x64x32 lattice with |lambda| <= 0.23 from the
    oracle's own ChebFD run (tests/golden/make_window_c2.py)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "ti_64x64x32_V1_seed1_window0.23.txt")
    return np.loadtxt(path)[:, 0]


def test_solve_full_size(env, orc):
    """The benchmark's solve (SELL-32-256, FP64, N_S 256, window holding 64
    eigenvalues): the 64 eigenvalues equal, one by one, those the oracle's
    own ChebFD run found in the window (to 1e-10 S_w, with the oracle's
    next eigenvalue outside the window); every returned pair has a
    residual <= 1e-9 when the oracle recomputes H v - lambda v, the vectors
    are orthonormal, the eigenvalues come in Kramers pairs, the matrix-free
    storage finds the same eigenvalues, and the precision form's complex64
    sweep, before its FP64 polish, has them all to 1e-5 S_w."""
    torch, B, ctx, Hr = env
    d = W["delta"]
    out = {}
    for storage, prec in (("sell", B.PREC_C128), ("stencil", B.PREC_C128),
                          ("sell", B.PREC_C64)):
        H = _matrix(B, ctx, storage)
        info = H.info()
        a, b = info["g_lo"], info["g_hi"]
        dp = d * (math.sqrt(W["n_s"] / W["n_target"]) - 1.0)
        n_p, _ = B.chebfd_optimal_np(a, b, -d, d, -d - dp, d + dp)
        p = B.default_params(lam_lo=-d, lam_hi=d, n_s=W["n_s"], n_p=n_p, kernel=W["kernel"],
                             mu=W["mu"], eps=W["eps"], max_iter=60, lock=1, precision=prec,
                             seed=W["seeds"][0],
                             vectors=1 if (storage == "sell" and prec == B.PREC_C128) else 0)
        out[(storage, prec)] = B.chebfd_solve(ctx, H, p)
        del H
        torch.cuda.empty_cache()
    rc, ev, rs, V, stats = out[("sell", B.PREC_C128)]
    S_w = max(abs(stats["a"]), abs(stats["b"]))
    assert rc == 0, stats
    assert ev.size == W["n_target"]
    gold = np.sort(_oracle_window())
    want = gold[np.abs(gold) <= d]
    assert want.size == ev.size and np.abs(gold[np.abs(gold) > d]).min() > d
    assert np.abs(ev - want).max() < 1e-10 * S_w
    assert np.all(np.abs(ev) <= d) and np.all(np.diff(ev) >= 0)
    # residuals recomputed by the reference's own sparse product
    HV = orc.spmm(Hr, V)
    r = np.linalg.norm(HV - V * ev, axis=0)
    assert r.max() <= 1e-9, r.max()
    assert np.abs(r - rs).max() < 1e-11
    G = V.conj().T @ V
    assert np.abs(G - np.eye(ev.size)).max() < 1e-10
    # time-reversal symmetry: exact Kramers pairs
    assert np.abs(ev[0::2] - ev[1::2]).max() < 1e-10 * S_w
    rc2, ev2, rs2, _, _ = out[("stencil", B.PREC_C128)]
    assert rc2 == 0 and ev2.size == ev.size
    assert np.abs(ev2 - ev).max() < 1e-10 * S_w
    assert rs2.max() <= 1e-9
    rc3, ev3, rs3, _, st3 = out[("sell", B.PREC_C64)]
    assert rc3 == 0 and ev3.size == ev.size
    assert np.abs(ev3 - want).max() < 1e-10 * S_w
    assert rs3.max() <= 1e-9
    sw = st3["sweep_evals"]
    assert sw.size == want.size, sw.size
    err32 = np.abs(sw - want).max() / S_w
    assert err32 < 1e-5, err32
    print(f"64x64x32 complex64 sweep: {sw.size} pairs, eigenvalue error {err32:.2e} S_w, "
          f"residuals up to {st3['sweep_residuals'].max():.1e}")


def test_precision_form_solve_128x128x64(orc):
    """The precision form at its full size (128x128x64, N = 4,194,304, N_S
    256, complex64 sweep + FP64 polish, 40-step Lanczos interval, window of
    half-width 0.1335 holding about 100 eigenvalues): every returned pair
    has a residual <= 1e-9 when the reference recomputes H v - lambda v with
    its own sparse product, the vectors are orthonormal, the eigenvalues
    lie in the window and come in Kramers pairs, and they are the FP64
    form's eigenvalues (same count, 1e-10 S_w); before the polish the
    complex64 sweep has them to 1e-5 S_w."""
    import torch
    from paper_1510_04895_amd import binding as B
    W3 = inp.WORKLOADS["ti_128x128x64"]
    ctx = B.Context(0)
    H = B.Matrix.ti(ctx, W3["L"], pbc=W3["pbc"], V=W3["V"], seed=W3["seeds"][0],
                    storage=B.STORAGE_STENCIL)
    a, b = B.chebfd_lanczos_bounds(ctx, H, k=40, seed=W3["seeds"][0])
    d = 0.1335
    dp = d * (math.sqrt(W3["n_s"] / W3["n_target"]) - 1.0)
    n_p, _ = B.chebfd_optimal_np(a, b, -d, d, -d - dp, d + dp)
    p = B.default_params(lam_lo=-d, lam_hi=d, n_s=W3["n_s"], n_p=n_p, kernel=W3["kernel"],
                         mu=W3["mu"], eps=W3["eps"], max_iter=40, lock=1,
                         precision=B.PREC_C64, seed=W3["seeds"][0], vectors=1, bounds=40)
    rc, ev, rs, V, stats = B.chebfd_solve(ctx, H, p)
    p.precision = B.PREC_C128
    p.vectors = 0
    rc64, ev64, rs64, _, st64 = B.chebfd_solve(ctx, H, p)
    del H
    torch.cuda.empty_cache()
    assert rc == 0, stats
    assert rc64 == 0, st64
    assert 90 <= ev.size <= 110 and ev.size % 2 == 0, ev.size
    S_w = max(abs(stats["a"]), abs(stats["b"]))
    assert ev64.size == ev.size and np.abs(ev64 - ev).max() < 1e-10 * S_w
    assert rs64.max() <= 1e-9
    sw = stats["sweep_evals"]
    nearest = np.abs(sw[:, None] - ev64[None, :]).min(axis=1)
    err32 = nearest.max() / S_w
    assert sw.size >= 0.9 * ev64.size and err32 < 1e-5, (sw.size, err32)
    print(f"128x128x64 complex64 sweep: {sw.size} of {ev64.size} pairs below sqrt(eps), "
          f"eigenvalue error {err32:.2e} S_w against the FP64 form; solve {stats['t_total']:.1f} s "
          f"(FP64 form {st64['t_total']:.1f} s)")
    assert np.all(np.abs(ev) <= d) and np.all(np.diff(ev) >= 0)
    assert np.abs(ev[0::2] - ev[1::2]).max() < 1e-10 * S_w
    Hr = orc.ti_hamiltonian(*W3["L"], pbc=W3["pbc"], V=W3["V"], seed=W3["seeds"][0])
    HV = orc.spmm(Hr, V)
    r = np.linalg.norm(HV - V * ev, axis=0)
    assert r.max() <= 1e-9, r.max()
    assert np.abs(r - rs).max() < 1e-11
    G = V.conj().T @ V
    assert np.abs(G - np.eye(ev.size)).max() < 1e-10


def test_adaptive_degree_full_size(env, orc):
    """The throughput configuration with the adaptive degree, started from
    N_p = 100: after the first pass the degree is re-selected from the
    256-vector density estimate, and the solve returns the oracle's 64
    window eigenvalues to 1e-10 S_w."""
    torch, B, ctx, Hr = env
    d = W["delta"]
    H = _matrix(B, ctx, "stencil")
    p = B.default_params(lam_lo=-d, lam_hi=d, n_s=W["n_s"], n_p=100, kernel=W["kernel"],
                         mu=W["mu"], eps=W["eps"], max_iter=60, lock=1, seed=W["seeds"][0],
                         vectors=0, adapt=1)
    rc, ev, rs, _, stats = B.chebfd_solve(ctx, H, p)
    del H
    torch.cuda.empty_cache()
    gold = np.sort(_oracle_window())
    want = gold[np.abs(gold) <= d]
    S_w = max(abs(stats["a"]), abs(stats["b"]))
    assert rc == 0 and ev.size == want.size, (rc, ev.size, stats)
    assert np.abs(ev - want).max() < 1e-10 * S_w
    assert rs.max() <= 1e-9
    # 201 moments resolve the density only to ~pi S_w / 201 = 0.13, wider than
    # the window, so the count of a density rising away from the gap is high
    assert 32 <= stats["n_t_estimate"] <= 128 and stats["n_p_used"] != 100, stats
    print(f"64x64x32 adaptive: n_p 100 -> {stats['n_p_used']}, N_T estimate "
          f"{stats['n_t_estimate']:.1f}, {stats['iterations']} iterations, "
          f"{stats['t_total']:.2f} s")


def test_random_block_and_convert_beyond_2_32_elements(env, orc):
    """Blocks of more than 2^32 entries (here (2^25 + 3) x 128 complex64,
    34 GB, then its complex128 copy, 69 GB): a dispatch holds fewer than
    2^32 work-items, so the element-wise kernels stride over a capped grid.
    Rows at the start, around 2^24 and at the end equal the reference
    generator bit for bit, before and after the conversion."""
    torch, B, ctx, _ = env
    torch.cuda.empty_cache()
    n, n_s, seed = (1 << 25) + 3, 128, 17
    assert n * n_s > 2**32
    X = torch.empty((n, n_s), dtype=torch.complex64, device="cuda")
    B.chebfd_random_block(ctx, X, seed=seed)
    Y = torch.empty((n, n_s), dtype=torch.complex128, device="cuda")
    B.chebfd_convert(ctx, X, Y)
    torch.cuda.synchronize()
    try:
        for i0 in (0, (1 << 24) - 1, (1 << 25) - 1, n - 2):
            ref = orc.random_block(2, n_s, seed=seed, stream=1, offset=i0 * n_s)
            got = X[i0:i0 + 2].cpu().numpy()
            assert np.array_equal(got, ref.astype(np.complex64)), i0
            assert np.array_equal(Y[i0:i0 + 2].cpu().numpy(), got.astype(np.complex128)), i0
    finally:
        del X, Y
        torch.cuda.empty_cache()


@pytest.mark.parametrize("storage,prec", [("stencil", "c128"), ("stencil", "c64"),
                                          ("sell", "c128")])
def test_filter_sampled_rows_at_256x256x64(orc, storage, prec):
    """The largest lattice in the benchmark's launch configurations
    (matrix-free: tiled lattice order with its XCD placement, 32 lanes per
    site in complex128, a whole wave per site in complex64; SELL-32-256:
    row groups of 4 in the tiled row order; 128 columns):
    a degree-3 filter, all of whose steps are fused launches, equals the
    reference at sampled rows.  Those include the lattice corners, the
    open z faces, the periodic wraps and the strip boundaries of the
    tiled order.  The reference evaluates the filter there from its own
    sparse rows and the input rows within three hops."""
    import torch
    from paper_1510_04895_amd import binding as B
    from sampled import sampled_filter
    torch.cuda.empty_cache()
    L, n_s, seed = (256, 256, 64), 128, 31
    Hr = orc.ti_hamiltonian(*L, pbc=3, V=1.0, seed=1)
    a, b = orc.gershgorin(Hr)
    gam = inp.random_gamma(3, seed=6)
    ctx = B.Context(0)
    H = B.Matrix.ti(ctx, L, pbc=3, V=1.0, seed=1,
                    storage=B.STORAGE_STENCIL if storage == "stencil" else B.STORAGE_SELL)
    dt = torch.complex128 if prec == "c128" else torch.complex64
    X = torch.empty((Hr.n, n_s), dtype=dt, device="cuda")
    B.chebfd_random_block(ctx, X, seed=seed)
    U, W = torch.empty_like(X), torch.empty_like(X)
    B.chebfd_filter_apply(ctx, H, gam, a, b, X, U, W)
    torch.cuda.synchronize()
    del U, W
    # sites: corners, open z faces, wraps, strip boundaries (x = 3, 4, 7,
    # 8, 251, 252), and seeded random ones
    Lx, Ly, Lz = L
    pick = [(0, 0, 0), (Lx - 1, Ly - 1, Lz - 1), (3, 0, 1), (4, Ly - 1, 62), (7, 128, 0),
            (8, 128, Lz - 1), (251, 5, 31), (252, 250, 32), (Lx - 1, 0, 33), (0, Ly - 1, 2)]
    g = np.random.default_rng(7)
    pick += [tuple(int(v) for v in g.integers(0, [Lx, Ly, Lz])) for _ in range(40)]
    sites = [x + Lx * (y + Ly * z) for x, y, z in pick]
    rows = [4 * s + o for s in sites for o in range(4)]

    def xrows(idx):
        # the input block: the reference generator's rows (rounded to
        # complex64 as the library's complex64 block holds them)
        out = np.concatenate([orc.random_block(1, n_s, seed=seed, stream=1, offset=int(r) * n_s)
                              for r in idx])
        return out.astype(np.complex64).astype(np.complex128) if prec == "c64" else out

    got_rows, ref = sampled_filter(Hr, a, b, gam, rows, xrows)
    got = X[torch.as_tensor(got_rows, device="cuda")].cpu().numpy().astype(np.complex128)
    del X, H
    torch.cuda.empty_cache()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    tol = 1e-12 * 3 if prec == "c128" else 30 * math.sqrt(3) * 2.0 ** -24
    assert err < tol, err
