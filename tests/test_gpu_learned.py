"""GPU parity of the learned form's pieces: KPM moments (fused kernel in
moment mode) and the network's forward, backward and Adam kernels, each
against the FP64 CPU reference on the same inputs."""
import numpy as np
import pytest

import chebfd_inputs as inp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1510_04895_amd import binding as B
    return torch, B, B.Context(0)


@pytest.mark.parametrize("prec,tol", [("c128", 1e-11), ("c64", 2e-5)])
def test_kpm_moments_vs_reference(env, orc, prec, tol):
    """mu_m = (1/(N R)) sum_r <x_r, T_m x_r> with the library's own random
    phases e^{2 pi i u} (u: stream 2 of the seed); the reference builds the
    same phases from its own generator and computes the moments directly."""
    torch, B, ctx = env
    L, R, M, seed = (5, 4, 3), 6, 40, 11
    Hr = orc.ti_hamiltonian(*L, pbc=3, V=1.0, seed=2)
    a, b = orc.gershgorin(Hr)
    H = B.Matrix.ti(ctx, L, pbc=3, V=1.0, seed=2)
    got = B.chebfd_kpm_moments(ctx, H, R, M, seed, a, b,
                               precision=B.PREC_C128 if prec == "c128" else B.PREC_C64)
    u = np.array([orc.u01(seed, 2, k) for k in range(Hr.n * R)]).reshape(Hr.n, R)
    X = np.exp(2j * np.pi * u)
    ref = orc.moments_direct(Hr, a, b, X, M).sum(1) / (Hr.n * R)
    assert np.abs(got - ref).max() < tol * max(1.0, np.abs(ref).max()) * M


@pytest.fixture(scope="module")
def net(env):
    torch, B, ctx = env
    n_in, h, n_out, Bsz = 20, 16, 6, 9
    mlp = B.MLP(ctx, n_in, h, n_out, seed=3)
    g = np.random.default_rng(4)
    X = g.normal(size=(Bsz, n_in)).astype(np.float32)
    T = g.normal(size=(Bsz, n_out)).astype(np.float32)
    shift = g.normal(size=n_out).astype(np.float32)
    scale = g.uniform(0.5, 2, n_out).astype(np.float32)
    mlp.set(shift=shift, scale=scale)
    ish = g.normal(size=n_in).astype(np.float32)
    isc = g.uniform(0.5, 2, n_in).astype(np.float32)
    mlp.input_scaling(ish, isc)
    return mlp, X, T, shift, scale, (n_in, h, n_out), ish, isc


def test_mlp_forward_vs_reference(env, net):
    from oracle import mlp as ref
    torch, B, ctx = env
    mlp, X, T, shift, scale, dims, ish, isc = net
    p, sh, sc = mlp.get()
    Y = mlp.forward(torch.from_numpy(X).cuda()).cpu().numpy()
    raw, _ = ref.forward(p.astype(np.float64), X.astype(np.float64), *dims, ish, isc)
    assert np.abs(Y - (raw * sc + sh)).max() < 1e-5 * max(1.0, np.abs(raw).max())


def test_mlp_gradient_vs_reference(env, net):
    from oracle import mlp as ref
    torch, B, ctx = env
    mlp, X, T, shift, scale, dims, ish, isc = net
    p, _, _ = mlp.get()
    loss, g = mlp.loss_grad(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda())
    lr, gr = ref.loss_grad(p, X, T, shift.astype(np.float64), scale.astype(np.float64), *dims,
                           ish.astype(np.float64), isc.astype(np.float64))
    assert loss == pytest.approx(lr, rel=1e-5)
    assert np.abs(g - gr).max() < 1e-5 * np.abs(gr).max()


def test_mlp_adam_steps_vs_reference(env, orc):
    """Three Adam steps on the device equal three reference steps."""
    from oracle import mlp as ref
    torch, B, ctx = env
    dims = (12, 10, 4)
    mlp = B.MLP(ctx, *dims, seed=9)
    g = np.random.default_rng(1)
    X = g.normal(size=(7, dims[0])).astype(np.float32)
    T = g.normal(size=(7, dims[2])).astype(np.float32)
    p, sh, sc = mlp.get()
    p = p.astype(np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    for step in range(1, 4):
        mlp.train_step(Xd, Td, lr=1e-3, weight_decay=1e-4)
        _, gr = ref.loss_grad(p, X, T, sh.astype(np.float64), sc.astype(np.float64), *dims)
        p, m, v = ref.adam_step(p, gr, m, v, step, 1e-3, 1e-4)
    pd, _, _ = mlp.get()
    assert np.abs(pd - p).max() < 2e-5


def test_mlp_training_reduces_loss(env):
    torch, B, ctx = env
    mlp = B.MLP(ctx, 8, 32, 3, seed=2)
    g = np.random.default_rng(5)
    X = g.normal(size=(64, 8)).astype(np.float32)
    W = g.normal(size=(8, 3)).astype(np.float32)
    T = np.tanh(X @ W).astype(np.float32)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    first = mlp.train_step(Xd, Td, lr=3e-3)
    for _ in range(400):
        last = mlp.train_step(Xd, Td, lr=3e-3)
    assert last < 0.05 * first


@pytest.mark.parametrize("seed", [10001, 10017])
def test_trained_model_on_heldout_realisation(env, seed):
    """The committed network on a held-out 32x32x16 realisation (seeds of
    the evaluation set, never trained on): its (N_p, N_S, corrections),
    gated by the damping-factor check, reach the same eigenvalues as the
    DOS rule's parameters at residual <= 1e-9.

    The network does not beat the rule.  On the 20 held-out realisations it
    needs 1.5% more matrix-vector products in total than the rule (median
    1.12x per realisation, range 0.85x-1.39x).  On the training sweep the
    rule is the best fixed point of the (N_S, N_p) grid, and the best point
    per realisation would save 12%, which the KPM features do not predict.
    The work bound is only a guard against a broken network or decoding."""
    import os
    torch, B, ctx = env
    from paper_1510_04895_amd import learned
    path = os.path.join(os.path.dirname(learned.__file__), "models", "ti_32x32x16_mlp.npz")
    net = learned.load_model(ctx, path)
    P = learned.problem(ctx, seed)
    base = learned.run_solve(ctx, P["H"], P["delta"], P["ns0"], P["np0"], seed=seed)
    n_p, n_s, corr = learned.predict(ctx, net, P)
    lrn = learned.run_solve(ctx, P["H"], P["delta"], n_s, n_p, corr=corr, seed=seed)
    S_w = max(abs(P["a"]), abs(P["b"]))
    assert base["rc"] == 0 and lrn["rc"] == 0
    assert lrn["found"] == base["found"]
    if base["found"]:
        assert np.abs(lrn["evals"] - base["evals"]).max() < 1e-10 * S_w
        assert lrn["res"].max() <= 1e-9
    assert lrn["n_mvm"] <= 1.5 * base["n_mvm"]
