"""Pins of the oracle's filter, dense algebra and ChebFD driver.

Each check compares against an independent definition: the scalar polynomial
on exact eigenpairs (Eq. (filterOne)), LAPACK via numpy, closed-form moments,
brute force on small inputs, or the paper's own numerical examples.
"""
import math

import numpy as np
import pytest

import chebfd_inputs as inp


def test_filter_diagonal_is_scalar_polynomial(orc):
    """Fig. fig:ChebFD on H = diag(lambda): Y_ik = p(lambda_i) X_ik with p
    evaluated point by point (Eq. (filterOne))."""
    lam = inp.flat_spectrum(300)
    H = orc.diagonal_csr(lam)
    X = inp.random_block(300, 5, seed=11)
    for n_p in [2, 3, 17, 200]:
        gam = inp.random_gamma(n_p, seed=n_p)
        Y = orc.filter_block(H, -1.0, 1.0, gam, X)
        p = np.array([orc.poly_eval(gam, -1.0, 1.0, l) for l in lam])
        assert np.abs(Y - p[:, None] * X).max() < 1e-12


def test_filter_on_ti_eigenvectors(orc):
    """p(H) v = p(lambda) v on exact eigenvectors of a 4x4x4 TI lattice (dense
    eigenvectors from LAPACK)."""
    H = orc.ti_hamiltonian(4, 4, 4, pbc=3, V=1.0, seed=5)
    a, b = orc.gershgorin(H)
    w, V = np.linalg.eigh(H.dense())
    idx = [0, 17, 128, 129, 255]
    gam = orc.gamma(-0.5, 0.5, a, b, 120, "lanczos")
    Y = orc.filter_block(H, a, b, gam, V[:, idx])
    p = np.array([orc.poly_eval(gam, a, b, w[i]) for i in idx])
    assert np.abs(Y - V[:, idx] * p[None, :]).max() < 1e-11


def test_filter_invalid_degree(orc):
    H = orc.diagonal_csr([0.1, 0.2])
    with pytest.raises(ValueError):
        orc.filter_block(H, -1, 1, np.array([1.0, 0.5]), np.ones((2, 1)))


def test_moments_direct_closed_form_diagonal(orc):
    """mu_m = sum_i |x_i|^2 T_m(alpha lambda_i + beta) on a diagonal matrix."""
    lam = inp.linear_spectrum(400) * 0.9
    H = orc.diagonal_csr(lam)
    X = inp.random_block(400, 3, seed=4)
    a, b = -1.3, 1.1
    mom = orc.moments_direct(H, a, b, X, 50)
    y = 2 / (b - a) * lam + (a + b) / (a - b)
    ref = np.array([(np.abs(X) ** 2 * np.cos(m * np.arccos(y))[:, None]).sum(0) for m in range(50)])
    assert np.abs(mom - ref).max() < 1e-10 * np.abs(ref).max()


def test_moments_doubling_matches_direct(orc):
    """Moments gathered during the filter from <T_n x, T_n x> and
    <T_{n-1} x, T_n x> (doubling) equal the direct <x, T_m x>, m = 0..2N_p."""
    H = orc.ti_hamiltonian(4, 4, 2, pbc=3, V=1.0, seed=9)
    a, b = orc.gershgorin(H)
    X = inp.random_block(H.n, 4, seed=3)
    n_p = 30
    _, mom = orc.filter_block(H, a, b, inp.random_gamma(n_p, 1), X, moments=True)
    ref = orc.moments_direct(H, a, b, X, 2 * n_p + 1)
    assert np.abs(mom - ref).max() < 1e-11 * np.abs(ref[0]).max()


def test_gram_kahan_vs_lapack(orc):
    A = inp.random_block(5000, 7, seed=1)
    B = inp.random_block(5000, 9, seed=2)
    S = orc.gram_kahan(A, B)
    assert np.abs(S - A.conj().T @ B).max() < 1e-10


def test_jacobi_vs_lapack(orc):
    g = np.random.default_rng(3)
    for n in [1, 2, 7, 40]:
        M = g.normal(size=(n, n)) + 1j * g.normal(size=(n, n))
        A = M + M.conj().T
        w, V = orc.jacobi_herm(A)
        assert np.abs(w - np.linalg.eigvalsh(A)).max() < 1e-12 * max(1, np.abs(w).max())
        assert np.abs(A @ V - V * w).max() < 1e-12 * np.abs(w).max()
        assert np.abs(V.conj().T @ V - np.eye(n)).max() < 1e-13
    # degenerate spectrum (Kramers pairs of a TI lattice)
    H = orc.ti_hamiltonian(2, 2, 4, pbc=3, V=1.0, seed=1)
    A = H.dense()
    w, V = orc.jacobi_herm(A)
    assert np.abs(w - np.linalg.eigvalsh(A)).max() < 1e-12
    assert np.abs(A @ V - V * w).max() < 1e-12


def test_svqb_orthonormal_same_span(orc):
    Y = inp.random_block(3000, 12, seed=7)
    Y[:, 3] *= 1e-6                               # poorly scaled column
    Q, nref = orc.svqb(Y)
    assert nref == 0
    assert np.abs(Q.conj().T @ Q - np.eye(12)).max() < 1e-13
    Pq = Q @ Q.conj().T
    Qy, _ = np.linalg.qr(Y)
    assert np.abs(Pq - Qy @ Qy.conj().T).max() < 1e-11


def test_svqb_rank_drop_refill(orc):
    """Linearly dependent columns are dropped and replaced by random vectors
    (Sec. 3.1, step 6 remarks); the result is still orthonormal and contains
    the original span."""
    Y = inp.random_block(2000, 8, seed=8)
    Y[:, 5] = Y[:, 1] * (0.5 - 0.25j)
    Y[:, 7] = 0.0
    Q, nref = orc.svqb(Y, seed=3)
    assert nref == 2
    assert np.abs(Q.conj().T @ Q - np.eye(8)).max() < 1e-13
    Yk = Y[:, [0, 1, 2, 3, 4, 6]]
    assert np.abs(Yk - Q @ (Q.conj().T @ Yk)).max() < 1e-12


def test_rayleigh_ritz_exact_invariant_subspace(orc):
    """An orthonormal basis of an exact invariant subspace returns its
    eigenvalues with zero residual (Sec. 3.1, step 7)."""
    H = orc.ti_hamiltonian(4, 4, 2, pbc=3, V=1.0, seed=2)
    w, V = np.linalg.eigh(H.dense())
    sel = [40, 41, 42, 43, 60, 61]
    g = np.random.default_rng(1)
    Q, _ = np.linalg.qr(g.normal(size=(6, 6)) + 1j * g.normal(size=(6, 6)))
    th, Vr, res = orc.rayleigh_ritz(H, V[:, sel] @ Q)
    assert np.abs(th - w[sel]).max() < 1e-12
    assert res.max() < 1e-12


def test_solve_diagonal_d1000(orc):
    """Sec. 3.2 example: D = 1000 equidistant eigenvalues, I_T = [-0.01,
    0.01] (N_T = 10), N_S = 50, N_p = 200, eps = 1e-7: all ten found."""
    lam = inp.flat_spectrum(1000)
    H = orc.diagonal_csr(lam)
    st, ev, res, V, stats = orc.chebfd_solve(H, -0.01, 0.01, 50, 200, eps=1e-7, seed=1,
                                              a=-1.0, b=1.0)
    assert st == 0
    want = lam[np.abs(lam) <= 0.01]
    assert want.size == 10 and ev.size == 10
    assert np.abs(ev - want).max() < 1e-12
    assert res.max() <= 1e-7
    # residuals recomputed from the returned vectors
    r = np.linalg.norm(lam[:, None] * V - V * ev[None, :], axis=0)
    assert r.max() <= 1e-7 * 1.01


def test_one_filter_step_weights(orc):
    """Fig. fig:filtermatrix case (ii): one Lanczos(mu=2) filter step with
    N_p = 200 and N_S = 50 on D = 1000 gives residual weight 1 - w_i <= 1.5e-5
    for the N_T = 10 target eigenvectors (Eq. (weight1)); allow a factor 3
    for the random start."""
    lam = inp.flat_spectrum(1000)
    H = orc.diagonal_csr(lam)
    gam = orc.gamma(-0.01, 0.01, -1, 1, 200, "lanczos")
    X = orc.random_block(1000, 50, seed=2)
    Y = orc.filter_block(H, -1, 1, gam, X)
    Q, _ = orc.svqb(Y)
    w = np.sqrt((np.abs(Q) ** 2).sum(1))        # eigenvectors are unit vectors e_i
    tgt = np.abs(lam) <= 0.01
    assert (1 - w[tgt]).max() <= 3 * 1.5e-5
    # case (i): N_S = N_T = 10 is far worse
    Y1 = orc.filter_block(H, -1, 1, gam, orc.random_block(1000, 10, seed=2))
    Q1, _ = orc.svqb(Y1)
    w1 = np.sqrt((np.abs(Q1) ** 2).sum(1))
    assert (1 - w1[tgt]).max() > 1e-3


def test_solve_ti_4x4x4_vs_dense(orc):
    """Full scheme on a 4x4x4 TI lattice against dense eigenvalues."""
    H = orc.ti_hamiltonian(4, 4, 4, pbc=3, V=1.0, seed=1)
    w = np.linalg.eigvalsh(H.dense())
    aw = np.sort(np.abs(w))
    d = 0.5 * (aw[3] + aw[4])                         # 4 eigenvalues in window
    st, ev, res, V, stats = orc.chebfd_solve(H, -d, d, 16, 60, eps=1e-9, seed=3)
    want = w[np.abs(w) <= d]
    assert st == 0 and ev.size == want.size == 4
    a, b = stats["a"], stats["b"]
    assert np.abs(ev - want).max() < 1e-10 * max(abs(a), abs(b))
    A = H.dense()
    assert np.linalg.norm(A @ V - V * ev, axis=0).max() <= 1e-9


@pytest.mark.slow
def test_table_num_linear_iterations_scaled(orc):
    """Table tab:num, linear DOS row N_S = 200 (N_p = 303, eps = 1e-12, 5
    iterations), scaled down tenfold in D, N_T and N_S: D = 4000 with the
    same delta = 0.05 (N_T = D delta^2 = 10) and N_S/N_T = 2, so delta'/delta
    = 0.41 and sigma are unchanged and the iteration count must be 5 +- 1
    (plus the one confirming iteration the exit rule adds)."""
    lam = inp.linear_spectrum(4000)
    H = orc.diagonal_csr(lam)
    st, ev, res, _, stats = orc.chebfd_solve(H, -0.05, 0.05, 20, 303, eps=1e-12, seed=1,
                                              a=-1.0, b=1.0, vectors=False, max_iter=12)
    assert st == 0
    want = lam[np.abs(lam) <= 0.05]
    assert want.size == 10 and ev.size == 10
    assert np.abs(ev - want).max() < 1e-12
    assert 4 <= stats["iterations"] - 1 <= 6


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_golden_dense_spectra_vs_lapack(orc, seed):
    """The stored 8x8x8 spectra (written by the oracle's Jacobi) agree with
    LAPACK on the oracle's matrix, and come in exact Kramers pairs."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", f"ti_8x8x8_V1_seed{seed}_evals.txt")
    w = np.loadtxt(path)
    H = orc.ti_hamiltonian(8, 8, 8, pbc=3, V=1.0, seed=seed)
    wl = np.linalg.eigvalsh(H.dense())
    assert w.size == 2048
    assert np.abs(w - wl).max() < 1e-11
    assert np.abs(w[0::2] - w[1::2]).max() < 1e-11


def test_solve_empty_window_returns_nothing(orc):
    """A window that holds no eigenvalue (checked against LAPACK): the exit
    rule of Sec. 3.1 step 8 ends the run with no pair and status 0."""
    H = orc.ti_hamiltonian(4, 4, 4, pbc=3, V=1.0, seed=1)
    w = np.linalg.eigvalsh(H.dense())
    lo, hi = w.max() + 0.5, w.max() + 1.0
    st, ev, rs, V, stats = orc.chebfd_solve(H, lo, hi, 16, 60, seed=3, max_iter=20)
    assert st == 0 and ev.size == 0
    assert stats["iterations"] < 20


def test_harmonic_ritz_petrov_galerkin_condition(orc):
    """Harmonic Ritz pairs (Sec. 3.1 step 7 remarks, Sec. 6) of a random
    orthonormal block Y for the target tau satisfy the defining condition,
    written out here with numpy: for each returned unit vector y in span(Y)
    there is a xi with P^H ((H - tau) y - xi y) = 0, P = (H - tau) Y; rho is
    the Rayleigh quotient y^H H y, returned ascending, with the residual
    |H y - rho y|."""
    H = orc.ti_hamiltonian(3, 3, 4, pbc=3, V=1.0, seed=5)
    A = H.dense()
    g = np.random.default_rng(3)
    Y, _ = np.linalg.qr(g.normal(size=(H.n, 12)) + 1j * g.normal(size=(H.n, 12)))
    tau = 0.3
    rho, V, res = orc.harmonic_ritz(H, Y, tau)
    P = (A - tau * np.eye(H.n)) @ Y
    # V in span(Y) and unit columns
    assert np.abs(Y @ (Y.conj().T @ V) - V).max() < 1e-12
    assert np.abs(np.linalg.norm(V, axis=0) - 1).max() < 1e-12
    for j in range(V.shape[1]):
        y = V[:, j]
        py, pby = P.conj().T @ y, P.conj().T @ ((A - tau * np.eye(H.n)) @ y)
        xi = np.vdot(py, pby) / np.vdot(py, py)
        assert abs(xi.imag) < 1e-9 * abs(xi)
        assert np.linalg.norm(pby - xi * py) <= 1e-10 * np.linalg.norm(pby)
        assert abs(rho[j] - np.vdot(y, A @ y).real) < 1e-12
        assert abs(res[j] - np.linalg.norm(A @ y - rho[j] * y)) < 1e-12
    assert np.all(np.diff(rho) >= 0)


def test_harmonic_ritz_exact_invariant_subspace(orc):
    """On an exact invariant subspace the harmonic Ritz values are the
    eigenvalues, whatever the target."""
    H = orc.ti_hamiltonian(4, 4, 2, pbc=3, V=1.0, seed=2)
    w, V = np.linalg.eigh(H.dense())
    sel = [40, 41, 42, 43, 60, 61]
    g = np.random.default_rng(1)
    Q, _ = np.linalg.qr(g.normal(size=(6, 6)) + 1j * g.normal(size=(6, 6)))
    rho, Vr, res = orc.harmonic_ritz(H, V[:, sel] @ Q, 0.17)
    assert np.abs(rho - w[sel]).max() < 1e-12
    assert res.max() < 1e-12


def test_solve_ti_4x4x4_harmonic_vs_dense(orc):
    """The scheme with harmonic Ritz extraction returns the dense spectrum's
    window eigenvalues."""
    H = orc.ti_hamiltonian(4, 4, 4, pbc=3, V=1.0, seed=1)
    w = np.linalg.eigvalsh(H.dense())
    aw = np.sort(np.abs(w))
    d = 0.5 * (aw[3] + aw[4])
    st, ev, res, V, stats = orc.chebfd_solve(H, -d, d, 16, 60, eps=1e-9, seed=3, harmonic=True)
    want = w[np.abs(w) <= d]
    assert st == 0 and ev.size == want.size == 4
    a, b = stats["a"], stats["b"]
    assert np.abs(ev - want).max() < 1e-10 * max(abs(a), abs(b))
    assert np.linalg.norm(H.dense() @ V - V * ev, axis=0).max() <= 1e-9


def test_sampled_filter_equals_reference_filter(orc):
    """The sampled-row evaluation used by the full-size parity tests agrees
    with the reference's filter of the whole block on a small lattice,
    including open-boundary and periodic-wrap sites."""
    import chebfd_inputs as inp
    from sampled import sampled_filter
    Hr = orc.ti_hamiltonian(6, 5, 4, pbc=3, V=1.0, seed=3)
    a, b = orc.gershgorin(Hr)
    X = inp.random_block(Hr.n, 5, seed=4)
    gam = inp.random_gamma(3, seed=5)
    full = orc.filter_block(Hr, a, b, gam, X)
    rows = [0, 1, 3, 17, 55, Hr.n - 1, Hr.n - 4, 4 * 29 + 2]
    got_rows, got = sampled_filter(Hr, a, b, gam, rows, lambda idx: X[idx])
    assert np.abs(got - full[got_rows]).max() < 1e-13 * np.abs(full).max()
