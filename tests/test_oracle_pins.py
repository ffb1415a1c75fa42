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


@pytest.mark.parametrize("L,pbc,V,seed", [((4, 4, 4), 3, 1.0, 3), ((5, 4, 3), 3, 1.7, 9),
                                          ((3, 6, 2), 7, 0.4, 2)])
def test_ti_gershgorin_exact(orc, L, pbc, V, seed):
    """Gershgorin interval of Eq. (Ham) in closed form: row (n, o) has the
    diagonal m g0(o) + V_n (g0 = +1 for tau = 0, -1 for tau = 1) and, per
    existing neighbour along j, two off-diagonal entries of modulus t/2 (one
    from G0, one from Gj), so its radius is t times the number of existing
    neighbours: 2 per periodic direction of extent >= 3, and along an open
    direction 2 in the interior, 1 on a surface.  A periodic direction of
    extent 2 reaches the same site both ways: the two blocks add to -t G0
    (the Gj parts cancel), one entry of modulus t.  V_n = V (u_n - 1/2) with
    u_n the (separately pinned) counter hash of stream 0 at index n."""
    m, t = 2.0, 1.0
    H = orc.ti_hamiltonian(*L, pbc=pbc, t=t, m=m, V=V, seed=seed)
    lo, hi = math.inf, -math.inf
    for z in range(L[2]):
        for y in range(L[1]):
            for x in range(L[0]):
                n = x + L[0] * (y + L[1] * z)
                vn = V * (orc.u01(seed, 0, n) - 0.5)
                nb = 0
                for j, c in enumerate((x, y, z)):
                    if (pbc >> j) & 1:
                        nb += 2 if L[j] >= 3 else 1
                    else:
                        nb += (c > 0) + (c < L[j] - 1)
                lo = min(lo, -m + vn - t * nb)
                hi = max(hi, m + vn + t * nb)
    a, b = orc.gershgorin(H)
    assert a == pytest.approx(lo, abs=1e-14) and b == pytest.approx(hi, abs=1e-14)


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


# --------------------------------------------------------------------------
# filter quality (Sec. 2.3) in closed form
# --------------------------------------------------------------------------
def test_filter_quality_closed_forms(orc):
    """sigma = max |p| outside I_S / min |p| inside I_T on [a, b] = [-1, 1]:
    p = T_2 = 2x^2 - 1 with I_T = [-0.1, 0.1] has its smallest modulus
    0.98 at the target edges and modulus 1 at x = +-1, so sigma = 1/0.98 > 1
    (eta = inf); p = 1 - x^2 = (T_0 - T_2)/2 with I_S = [-0.5, 0.5] has 0.99
    inside and at most 0.75 outside (at the search edges), sigma = 0.75/0.99
    and eta = -2/log10(sigma);
    p = x^2 = (T_0 + T_2)/2 with I_T = [0.4, 0.6], I_S = [0.3, 0.7] gives
    0.16 inside and 1 at x = +-1 outside, sigma = 6.25 > 1 and eta = inf;
    p = T_3 = 4x^3 - 3x with I_T = [0.5, 0.6], I_S = [0.2, 0.8]: inside,
    T_3 rises from -1 at 0.5 towards its zero at sqrt(3)/2, so the smallest
    modulus is |T_3(0.6)| = 0.936; outside the largest modulus is 1 (x = +-1),
    sigma = 1/0.936.
    The second case scaled to [a, b] = [-3, 5] (lambda = 1 + 4x) is the
    same."""
    s, e = orc.filter_quality([0.0, 0.0, 1.0], -1, 1, -0.1, 0.1, -0.5, 0.5)
    assert s == pytest.approx(1 / 0.98, rel=1e-14) and e == math.inf
    s, e = orc.filter_quality([0.5, 0.0, -0.5], -1, 1, -0.1, 0.1, -0.5, 0.5)
    assert s == pytest.approx(0.75 / 0.99, rel=1e-14)
    assert e == pytest.approx(-2 / math.log10(0.75 / 0.99), rel=1e-12)
    s, e = orc.filter_quality([0.5, 0.0, 0.5], -1, 1, 0.4, 0.6, 0.3, 0.7)
    assert s == pytest.approx(6.25, rel=1e-14) and e == math.inf
    s, e = orc.filter_quality([0.0, 0.0, 0.0, 1.0], -1, 1, 0.5, 0.6, 0.2, 0.8)
    assert s == pytest.approx(1 / 0.936, rel=1e-13)
    s, e = orc.filter_quality([0.5, 0.0, 0.5], -3, 5, 2.6, 3.4, 2.2, 3.8)
    assert s == pytest.approx(6.25, rel=1e-14)


# --------------------------------------------------------------------------
# density of states from moments (Eq. DOS:target, Eq. DOS:search)
# --------------------------------------------------------------------------
def _exact_moments(lam, M, a, b):
    x = (2 * lam - a - b) / (b - a)
    return np.cos(np.outer(np.arange(M), np.arccos(x))).mean(1)


@pytest.mark.parametrize("spectrum", ["flat", "linear"])
def test_dos_count_and_margin_closed_forms(orc, spectrum):
    """Exact moments mu_m = (1/D) sum_i T_m(x_i) of a known spectrum: the
    KPM count of Eq. DOS:target over a window whose edges lie between
    eigenvalues is the true count within 1 (the kernel smears each edge
    symmetrically; 2048 moments resolve ~0.003, finer than the window); and
    the margin of Eq. DOS:search for N_S = 2 N_T is delta' = delta for a
    flat DOS (the search interval doubles) and (sqrt 2 - 1) delta for a DOS
    proportional to |lambda| (the count grows as the square of the
    half-width), within the KPM resolution."""
    D = 4000
    lam = inp.flat_spectrum(D) if spectrum == "flat" else inp.linear_spectrum(D)
    a, b = -1.05, 1.05
    mu = _exact_moments(lam, 2048, a, b)
    d = 0.25
    true = int((np.abs(lam) <= d).sum())
    nt = orc.dos_count(mu, D, a, b, -d, d)
    assert abs(nt - true) <= 1.0
    dp = orc.dos_margin(mu, D, a, b, -d, d, 2 * true)
    want = d if spectrum == "flat" else (math.sqrt(2) - 1) * d
    assert abs(dp - want) <= 4 * (b - a) / 2048
    # integrating the density itself gives the same count
    xs = np.linspace(-d, d, 20001)
    rho = orc.kpm_density(mu, a, b, xs)
    assert D * integrate.simpson(rho, x=xs) == pytest.approx(nt, rel=1e-4)
