"""Pins of the oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself by retyping its formulas: every
check is a printed value from the paper, a closed form, an independent
quadrature / library routine, an invariant, or a brute-force evaluation.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import chebfd_inputs as inp


# --------------------------------------------------------------------------
# counter-based random numbers
# --------------------------------------------------------------------------
def test_splitmix64_published_vectors(orc):
    """The mixing function is SplitMix64's finaliser.  Applied to the
    generator states seed + G*(i+1) it must reproduce the published output
    sequences (seed 0: 0xe220a8397b1dcdaf, 0x6e789e6aa1b965f4; seed 1234567:
    6457827717110365317, 3203168211198807973, 9817491932198370423), and
    orc_hash(seed, s, i) must be the two-level composition
    mix(mix(seed + G(s+1)) + G(i+1))."""
    import ctypes as C
    G = 0x9E3779B97F4A7C15
    M = (1 << 64) - 1
    L = orc.lib()
    L.orc_mix64_public.restype = C.c_uint64
    L.orc_mix64_public.argtypes = [C.c_uint64]
    mix = L.orc_mix64_public
    assert [mix((0 + G * (i + 1)) & M) for i in range(2)] == [0xE220A8397B1DCDAF,
                                                              0x6E789E6AA1B965F4]
    assert [mix((1234567 + G * (i + 1)) & M) for i in range(3)] == [
        6457827717110365317, 3203168211198807973, 9817491932198370423]
    k = mix((5 + G * 3) & M)
    assert orc.hash64(5, 2, 7) == mix((k + G * 8) & M)


def test_u01_range_and_moments(orc):
    u = np.array([orc.u01(3, 1, i) for i in range(20000)])
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.01
    assert abs(u.var() - 1 / 12) < 0.003
    # 53-bit grid
    assert np.all(u * 2.0**53 == np.floor(u * 2.0**53))


# --------------------------------------------------------------------------
# Chebyshev polynomials, coefficients and kernels (Sec. 2.1)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [0, 1, 2, 5, 40, 333])
def test_chebyshev_recurrence_is_cos(orc, n):
    """T_n(cos theta) = cos(n theta) through the three-term recurrence."""
    gam = np.zeros(max(n, 2) + 1)
    gam[n] = 1.0
    for th in np.linspace(0.0, math.pi, 37):
        lam = math.cos(th)           # [a, b] = [-1, 1]: alpha = 1, beta = 0
        assert abs(orc.poly_eval(gam, -1.0, 1.0, lam) - math.cos(n * th)) < 1e-12 * max(1, n)


@pytest.mark.parametrize("win,ab", [((-0.01, 0.01), (-1, 1)), ((0.3, 0.7), (-2.0, 1.5)),
                                    ((-1.2, -0.4), (-1.5, 3.0))])
def test_window_coeffs_match_quadrature(orc, win, ab):
    """c_n = (2 - delta_n0)/pi * int W T_n (1-x^2)^{-1/2} dx, evaluated by
    adaptive quadrature in theta (x = cos theta), independently of the
    closed form (and fixing its overall sign)."""
    lo, hi = win
    a, b = ab
    n_p = 60
    c = orc.window_coeffs(lo, hi, a, b, n_p)
    al, be = 2 / (b - a), (a + b) / (a - b)
    th_lo, th_hi = math.acos(al * lo + be), math.acos(al * hi + be)
    for n in range(n_p + 1):
        q, _ = integrate.quad(lambda t: math.cos(n * t), th_hi, th_lo, epsabs=1e-13, limit=200)
        ref = (2 - (n == 0)) / math.pi * q
        assert abs(c[n] - ref) < 1e-11
    assert c[0] > 0


def test_filter_tends_to_window(orc):
    """p(x) -> W(x) away from the edges as N_p grows (Eq. (W2)); the
    derived sign gives p(centre) -> +1."""
    for n_p, tol in [(2000, 2e-3), (20000, 1e-4)]:
        g = orc.gamma(-0.01, 0.01, -1, 1, n_p, "lanczos")
        assert abs(orc.poly_eval(g, -1, 1, 0.0) - 1.0) < tol
        assert abs(orc.poly_eval(g, -1, 1, 0.3)) < tol
    g = orc.gamma(-0.01, 0.01, -1, 1, 2000, "none")
    assert abs(orc.poly_eval(g, -1, 1, 0.0) - 1.0) < 0.03   # Gibbs ripple without a kernel


def test_kernels_closed_form_invariants(orc):
    n_p = 97
    for k in ["none", "fejer", "jackson", "lanczos"]:
        assert orc.kernel(k, n_p)[0] == pytest.approx(1.0, abs=1e-15)
    f = orc.kernel("fejer", n_p)
    assert np.allclose(np.diff(f), -1.0 / (n_p + 1))
    assert f[-1] == pytest.approx(1.0 / (n_p + 1))
    j = orc.kernel("jackson", n_p)
    # as printed (N_p in the denominators): g_{N_p-1} = g_{N_p} = 0
    assert abs(j[-1]) < 1e-14 and abs(j[-2]) < 1e-14
    assert np.all(np.diff(j) < 1e-15)                    # monotone decay
    lz = orc.kernel("lanczos", 2 * 50 - 1, mu=2.0)      # N_p + 1 = 100
    assert lz[50] == pytest.approx((math.sin(math.pi / 2) / (math.pi / 2)) ** 2, rel=1e-14)
    l3 = orc.kernel("lanczos", 99, mu=3.0)
    assert l3[50] == pytest.approx((2 / math.pi) ** 3, rel=1e-14)
    assert np.all(orc.kernel("none", 10) == 1.0)


# --------------------------------------------------------------------------
# filter quality and parameter rules (Secs. 2.3, 2.4, Tables 2 and 3)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("kind,printed", [("lanczos", 6251), ("jackson", 7899), ("none", 1424)])
def test_optimal_np_fig_polyeff1(orc, kind, printed):
    """delta = delta' = 1e-3 in [-1,1]: the paper prints N_p^opt =
    6251 / 7899 / 1424 for Lanczos(mu=2) / Jackson / no kernel."""
    n, eta = orc.optimal_np(-1, 1, -1e-3, 1e-3, -2e-3, 2e-3, kind=kind,
                            lo=printed // 2, hi=2 * printed)
    assert abs(n - printed) <= 0.005 * printed


@pytest.mark.parametrize("delta,ratio,np_pr,eta_pr", [
    (0.0025, 0.75, 3320, 1368), (0.0025, 1.00, 2500, 1023),
    (0.0025, 3.00, 817, 351), (0.0025, 5.00, 495, 235),
    (0.05, 0.12, 1037, 427), (0.05, 0.41, 303, 125),
    (0.05, 1.00, 124, 51), (0.05, 1.45, 85, 36)])
def test_table_num_optimal_np_eta(orc, delta, ratio, np_pr, eta_pr):
    """Table tab:num: optimal N_p and eta for the printed search margin
    delta'/delta (flat DOS rows delta = 0.0025, linear DOS rows delta =
    0.05); exhaustive search over N_0 in [1, 16].  N_p and eta scale as
    1/delta' (Eq. (etafit)), so the printed two-digit ratio carries a relative
    uncertainty 0.005/ratio that is added to a 1.5% model tolerance; printed
    eta values are rounded to integers (+-0.5)."""
    dp = ratio * delta
    n, eta = orc.optimal_np(-1, 1, -delta, delta, -delta - dp, delta + dp)
    rel = 0.015 + 0.005 / ratio
    assert abs(n - np_pr) <= max(2, rel * np_pr)
    assert abs(eta - eta_pr) <= 0.5 + rel * eta_pr


@pytest.mark.parametrize("c,N0,eta0", [(0.0, 6.23, 2.58), (0.5, 5.40, 2.24), (0.8, 3.75, 1.55)])
def test_table_lanczoskernel_fit_constants(orc, c, N0, eta0):
    """Table tab:lanczoskernel at delta/S_w = 1e-3 (delta' = delta): N_p^opt
    = N_0 S_w/delta' and eta^opt = eta_0 S_w/delta'.  Fit constants: 2%."""
    d = 1e-3
    n, eta = orc.optimal_np(-1, 1, c - d, c + d, c - 2 * d, c + 2 * d,
                            lo=int(N0 / d / 2), hi=int(2 * N0 / d))
    assert n * d == pytest.approx(N0, rel=0.02)
    assert eta * d == pytest.approx(eta0, rel=0.02)


def test_effort_models(orc):
    """Eq. (etanlinear) is minimal at N_S = 4 N_T with value 4; Eq. (etanflat)
    decreases monotonically towards 1; Table tab:num's estimate column is
    eta * N_S * 12 (epsilon = 1e-12)."""
    r = np.linspace(1.05, 20, 40000)
    el = orc.effort_linear(r)
    assert r[np.argmin(el)] == pytest.approx(4.0, abs=1e-3)
    assert el.min() == pytest.approx(4.0, abs=1e-6)
    ef = orc.effort_flat(r)
    assert np.all(np.diff(ef) < 0) and ef[-1] > 1.0
    assert 1023 * 200 * 12 / 1e6 == pytest.approx(2.45, abs=0.01)
    assert 51 * 400 * 12 / 1e6 == pytest.approx(0.24, abs=0.01)


def test_intensity_model_printed_forms(orc):
    """Sec. 4.2: I(n_b) = 146/(260/n_b + 80) (complex FP64, N_nzr=13) and
    19/(48/n_b + 40) (real FP64, N_nzr=4)."""
    for nb in [1, 2, 16, 64, 256]:
        assert orc.intensity(nb, 13, 2, 6, 16, 4) == pytest.approx(146 / (260 / nb + 80))
        assert orc.intensity(nb, 4, 1, 1, 8, 4) == pytest.approx(19 / (48 / nb + 40))


# --------------------------------------------------------------------------
# Topological-insulator Hamiltonian (Sec. 5.1, Eq. (Ham))
# --------------------------------------------------------------------------
def _periodic_spectrum(L, t=1.0, m=2.0):
    ks = [2 * np.pi * np.arange(n) / n for n in L]
    E = []
    for kx in ks[0]:
        for ky in ks[1]:
            for kz in ks[2]:
                e = math.sqrt((m - t * (math.cos(kx) + math.cos(ky) + math.cos(kz))) ** 2
                              + t * t * (math.sin(kx) ** 2 + math.sin(ky) ** 2 + math.sin(kz) ** 2))
                E += [e, e, -e, -e]
    return np.sort(E)


@pytest.mark.parametrize("L", [(4, 4, 4), (3, 5, 4), (6, 2, 3)])
def test_ti_periodic_closed_form_spectrum(orc, L):
    H = orc.ti_hamiltonian(*L, pbc=7, V=0.0)
    A = H.dense()
    assert np.abs(A - A.conj().T).max() == 0.0
    w = np.linalg.eigvalsh(A)
    assert np.abs(w - _periodic_spectrum(L)).max() < 1e-12


def test_ti_structure_and_disorder(orc):
    Lx, Ly, Lz = 6, 5, 4
    V = 1.0
    H = orc.ti_hamiltonian(Lx, Ly, Lz, pbc=3, V=V, seed=7)
    n = 4 * Lx * Ly * Lz
    rl = np.diff(H.rowptr)
    z = (np.arange(n) // 4) // (Lx * Ly)
    assert np.all(rl[(z > 0) & (z < Lz - 1)] == 13)     # 1 on-site + 6 hops x 2
    assert np.all(rl[(z == 0) | (z == Lz - 1)] == 11)   # open z surfaces
    assert H.nnz == pytest.approx(n * (13 - 4 / Lz))
    A = H.dense()
    d = np.real(np.diag(A))
    o = np.arange(n) % 4
    vn = d - np.where(o < 2, 2.0, -2.0)
    assert np.all(np.abs(vn) <= V / 2)
    # V_n is per site: the same for the 4 orbitals
    assert np.allclose(vn.reshape(-1, 4), vn.reshape(-1, 4)[:, :1], rtol=0, atol=1e-15)
    # off-diagonal entries have modulus 1/2
    off = A - np.diag(np.diag(A))
    nz = np.abs(off[off != 0])
    assert np.allclose(nz, 0.5)


def test_ti_kramers_pairs_and_gershgorin(orc):
    H = orc.ti_hamiltonian(4, 4, 4, pbc=3, V=1.0, seed=3)
    w = np.linalg.eigvalsh(H.dense())
    assert np.abs(w[0::2] - w[1::2]).max() < 1e-12        # Theta^2 = -1
    a, b = orc.gershgorin(H)
    assert a <= w[0] and w[-1] <= b
    assert b == pytest.approx(8.5, abs=0.5) and a == pytest.approx(-8.5, abs=0.5)


def test_ti_gauge_sign_of_hopping(orc):
    """t -> -t leaves the spectrum unchanged for even Lx, Ly (bipartite
    gauge), V = 0 and V != 0 alike."""
    for V in [0.0, 1.0]:
        w1 = np.linalg.eigvalsh(orc.ti_hamiltonian(4, 4, 3, pbc=3, t=1.0, V=V, seed=2).dense())
        w2 = np.linalg.eigvalsh(orc.ti_hamiltonian(4, 4, 3, pbc=3, t=-1.0, V=V, seed=2).dense())
        assert np.abs(w1 - w2).max() < 1e-12


def test_ti_small_periodic_duplicates_merge(orc):
    """Extent 2 along a periodic direction: the forward and backward hops hit
    the same site and are summed; the closed form still holds."""
    H = orc.ti_hamiltonian(2, 2, 2, pbc=7, V=0.0)
    w = np.linalg.eigvalsh(H.dense())
    assert np.abs(w - _periodic_spectrum((2, 2, 2))).max() < 1e-12
