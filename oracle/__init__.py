"""Plain CPU FP64 oracle for Chebyshev filter diagonalisation (ChebFD).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU library
(``paper_1510_04895_amd``) never imports it, and it never imports the GPU
library: the two share no code.  The only thing both sides consume is the
seeded input module ``chebfd_inputs``, which holds none of the method's
arithmetic.

The heavy parts are plain C (``chebfd_oracle.c``, FP64, -ffp-contract=off,
OpenMP static schedules) reached through ctypes; closed-form models from the
paper are plain Python below.  Each function names the passage it follows in
Pieper et al., arXiv:1510.04895.

Parity status: every function here is pinned by a ``-m "not gpu"`` test except
``mlp_*`` training dynamics (gradients are pinned by finite differences).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "chebfd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

KERNELS = {"none": 0, "fejer": 1, "jackson": 2, "lanczos": 3}


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (plain -O2, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
            "-ffp-contract=off", "-fno-fast-math", "-D_GNU_SOURCE",
            _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        i64, u64, i32, dbl, vp = C.c_int64, C.c_uint64, C.c_int, C.c_double, C.c_void_p
        L.orc_hash.restype = u64
        L.orc_hash.argtypes = [u64, u64, u64]
        L.orc_u01.restype = dbl
        L.orc_u01.argtypes = [u64, u64, u64]
        L.orc_random_block.argtypes = [i64, i64, u64, u64, u64, vp]
        L.orc_ti_max_nnz.restype = i64
        L.orc_ti_max_nnz.argtypes = [i32, i32, i32]
        L.orc_ti_csr.restype = i64
        L.orc_ti_csr.argtypes = [i32, i32, i32, i32, dbl, dbl, dbl, u64, vp, vp, vp]
        L.orc_gershgorin.argtypes = [i64, vp, vp, vp, vp, vp]
        L.orc_spmm.argtypes = [i64, vp, vp, vp, vp, vp, i64]
        L.orc_window_coeffs.argtypes = [dbl, dbl, dbl, dbl, i32, vp]
        L.orc_kernel.argtypes = [i32, i32, dbl, vp]
        L.orc_poly_eval.restype = dbl
        L.orc_poly_eval.argtypes = [vp, i32, dbl, dbl, dbl]
        L.orc_filter.restype = i32
        L.orc_filter.argtypes = [i64, vp, vp, vp, dbl, dbl, vp, i32, vp, vp, vp, i64, vp]
        L.orc_moments_direct.argtypes = [i64, vp, vp, vp, dbl, dbl, vp, i64, i32, vp]
        L.orc_gram_kahan.argtypes = [i64, vp, i64, vp, i64, vp]
        L.orc_block_times_small.argtypes = [i64, vp, i64, vp, i64, vp]
        L.orc_jacobi_herm.restype = i32
        L.orc_jacobi_herm.argtypes = [i32, vp, vp, vp]
        L.orc_svqb.restype = i32
        L.orc_svqb.argtypes = [i64, vp, vp, i64, dbl, u64, u64]
        L.orc_rayleigh_ritz.argtypes = [i64, vp, vp, vp, vp, vp, vp, i64, vp, vp]
        L.orc_chebfd_solve.restype = i32
        L.orc_harmonic_ritz.restype = i32
        L.orc_harmonic_ritz.argtypes = [i64, vp, vp, vp, vp, vp, vp, i64, dbl, vp, vp]
        L.orc_chebfd_solve.argtypes = [i64, vp, vp, vp, dbl, dbl, i64, i32, i32, dbl, dbl, i32,
                                       u64, dbl, dbl, vp, vp, vp, vp, i32]
        L.orc_num_threads.restype = i32
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


# --------------------------------------------------------------------------
# random numbers and inputs the method draws (Sec. 3.1 step 4, Sec. 5.1)
# --------------------------------------------------------------------------
def u01(seed: int, stream: int, index: int) -> float:
    return lib().orc_u01(seed, stream, index)


def hash64(seed: int, stream: int, index: int) -> int:
    return lib().orc_hash(seed, stream, index)


def random_block(n: int, n_s: int, seed: int, stream: int = 1, offset: int = 0) -> np.ndarray:
    X = np.empty((n, n_s), np.complex128)
    lib().orc_random_block(n, n_s, seed, stream, offset, _p(X))
    return X


class CSR:
    def __init__(self, n, rowptr, col, val):
        self.n, self.rowptr, self.col, self.val = n, rowptr, col, val

    @property
    def nnz(self):
        return int(self.rowptr[-1])

    def dense(self) -> np.ndarray:
        A = np.zeros((self.n, self.n), np.complex128)
        for i in range(self.n):
            for p in range(self.rowptr[i], self.rowptr[i + 1]):
                A[i, self.col[p]] += self.val[p]
        return A

    def ptrs(self):
        return (_p(self.rowptr), _p(self.col), _p(self.val))


def ti_hamiltonian(Lx, Ly, Lz, pbc=3, t=1.0, m=2.0, V=1.0, seed=1) -> CSR:
    """CSR of Eq. (Ham), Sec. 5.1; see chebfd_oracle.c for the conventions."""
    n = 4 * Lx * Ly * Lz
    cap = lib().orc_ti_max_nnz(Lx, Ly, Lz)
    rowptr = np.zeros(n + 1, np.int64)
    col = np.zeros(cap, np.int32)
    val = np.zeros(cap, np.complex128)
    nnz = lib().orc_ti_csr(Lx, Ly, Lz, pbc, t, m, V, seed, _p(rowptr), _p(col), _p(val))
    return CSR(n, rowptr, col[:nnz].copy(), val[:nnz].copy())


def csr_from_dense(A: np.ndarray) -> CSR:
    n = A.shape[0]
    rowptr = [0]
    cols, vals = [], []
    for i in range(n):
        nz = np.nonzero(A[i])[0]
        cols.extend(nz.tolist())
        vals.extend(A[i, nz].tolist())
        rowptr.append(len(cols))
    return CSR(n, np.array(rowptr, np.int64), np.array(cols, np.int32),
               np.array(vals, np.complex128))


def diagonal_csr(lams) -> CSR:
    lams = np.asarray(lams, np.float64)
    n = lams.size
    return CSR(n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32),
               lams.astype(np.complex128))


def gershgorin(H: CSR):
    a = C.c_double()
    b = C.c_double()
    lib().orc_gershgorin(H.n, *H.ptrs(), C.byref(a), C.byref(b))
    return a.value, b.value


def spmm(H: CSR, X: np.ndarray) -> np.ndarray:
    X = np.ascontiguousarray(X, np.complex128)
    Y = np.empty_like(X)
    lib().orc_spmm(H.n, *H.ptrs(), _p(X), _p(Y), X.shape[1])
    return Y


# --------------------------------------------------------------------------
# filter polynomials (Sec. 2.1, Table tab:Kernel) and their quality (Sec. 2.3)
# --------------------------------------------------------------------------
def window_coeffs(lam_lo, lam_hi, a, b, n_p) -> np.ndarray:
    c = np.empty(n_p + 1)
    lib().orc_window_coeffs(lam_lo, lam_hi, a, b, n_p, _p(c))
    return c


def kernel(kind, n_p, mu=2.0) -> np.ndarray:
    g = np.empty(n_p + 1)
    lib().orc_kernel(KERNELS[kind] if isinstance(kind, str) else kind, n_p, mu, _p(g))
    return g


def gamma(lam_lo, lam_hi, a, b, n_p, kind="lanczos", mu=2.0) -> np.ndarray:
    """gamma_n = g_n c_n, the coefficients of Eq. (W2)."""
    return window_coeffs(lam_lo, lam_hi, a, b, n_p) * kernel(kind, n_p, mu)


def poly_eval(gam, a, b, lam) -> float:
    gam = np.ascontiguousarray(gam, np.float64)
    return lib().orc_poly_eval(_p(gam), gam.size - 1, a, b, lam)


def filter_quality(gam, a, b, t_lo, t_hi, s_lo, s_hi, pts_per_period=16):
    """(sigma, eta) of Sec. 2.3: sigma = max |p| over [a, b] outside the
    search interval [s_lo, s_hi] divided by min |p| over the target
    [t_lo, t_hi], eta = -N_p / log10(sigma).  p is evaluated on the uniform
    theta grid theta_k = pi k / M (x = cos theta_k, pts_per_period points
    per period of T_{N_p}) by one type-I discrete cosine transform (a
    library FFT), p(cos theta_k) = sum_n gamma_n cos(n theta_k); the four
    interval edges are evaluated by the recurrence."""
    from scipy.fft import dct
    gam = np.asarray(gam, np.float64)
    n_p = gam.size - 1
    M = max(pts_per_period * (n_p + 1) // 2, n_p + 1)
    x = np.zeros(M + 1)
    x[:n_p + 1] = gam
    y = dct(x, type=1)
    p = np.abs(0.5 * (y + x[0]))
    th = np.pi * np.arange(M + 1) / M
    lam = a + (b - a) * 0.5 * (np.cos(th) + 1.0)
    inside = (lam >= t_lo) & (lam <= t_hi)
    outside = (lam < s_lo) | (lam > s_hi)
    mn = min(p[inside].min() if inside.any() else np.inf,
             abs(poly_eval(gam, a, b, t_lo)), abs(poly_eval(gam, a, b, t_hi)))
    mx = max(p[outside].max() if outside.any() else 0.0,
             abs(poly_eval(gam, a, b, s_lo)), abs(poly_eval(gam, a, b, s_hi)))
    sigma = mx / mn
    eta = -n_p / math.log10(sigma) if sigma < 1.0 else math.inf
    return sigma, eta


def eta_of_np(n_p, a, b, t_lo, t_hi, s_lo, s_hi, kind="lanczos", mu=2.0, pts=16):
    g = gamma(t_lo, t_hi, a, b, n_p, kind, mu)
    return filter_quality(g, a, b, t_lo, t_hi, s_lo, s_hi, pts)[1]


def optimal_np(a, b, t_lo, t_hi, s_lo, s_hi, kind="lanczos", mu=2.0, lo=None, hi=None, pts=16):
    """N_p minimising eta for the given interval configuration (Sec. 2.3,
    Sec. 3.1 step 3).  eta(N_p) is jagged (sidelobes crossing the search
    interval edge make local minima), so the search is exhaustive: every
    integer when the range is short, else a 0.2% geometric grid followed by
    an integer scan of +-1.5% around the three best grid points.  Default
    range: N_0 in [1, 16] in N_p = N_0 S_w / delta'."""
    S_w = 0.5 * (b - a)
    dp = max(min(t_lo - s_lo, s_hi - t_hi), 1e-300)
    if lo is None:
        lo = max(4, int(1.0 * S_w / dp))
    if hi is None:
        hi = int(16.0 * S_w / dp) + 8
    f = {}

    def ev(k):
        if k not in f:
            f[k] = eta_of_np(k, a, b, t_lo, t_hi, s_lo, s_hi, kind, mu, pts)
        return f[k]

    if hi - lo <= 2000:
        cand = range(lo, hi + 1)
        best = min(cand, key=ev)
        return best, ev(best)
    grid = sorted({int(round(lo * 1.002 ** i)) for i in range(int(math.log(hi / lo) / math.log(1.002)) + 2)})
    grid = [k for k in grid if lo <= k <= hi]
    top = sorted(grid, key=ev)[:3]
    for k in top:
        w = max(2, int(0.015 * k))
        for j in range(max(lo, k - w), min(hi, k + w) + 1):
            ev(j)
    best = min(f, key=lambda k: f[k])
    return best, f[best]


# density of states from KPM moments (Sec. 3.1 steps 1-3) --------------------
def kpm_density(mu, a, b, lam):
    """KPM estimate of the normalised DOS at lam (per unit lambda, integral
    1 over [a, b]) from moments mu_m = <T_m(alpha H + beta)>/D, m < M:
    rho(x) = [g_0 mu_0 + 2 sum_{m>=1} g_m mu_m T_m(x)] / (pi sqrt(1 - x^2))
    in the scaled variable x, with the Jackson factors of Table tab:Kernel
    at N_p = M (so g_{M-1} = 0), times dx/dlambda = 2/(b - a)."""
    mu = np.asarray(mu, np.float64)
    M = mu.size
    g = kernel("jackson", M)[:M]
    x = (2.0 * np.asarray(lam, np.float64) - a - b) / (b - a)
    th = np.arccos(np.clip(x, -1.0, 1.0))
    m = np.arange(1, M)
    s = g[0] * mu[0] + 2.0 * (g[1:] * mu[1:] * np.cos(np.multiply.outer(th, m))).sum(-1)
    return s / (np.pi * np.sqrt(1.0 - x * x)) * 2.0 / (b - a)


def dos_count(mu, D, a, b, lo, hi):
    """Eq. DOS:target with the KPM density: D times the integral of rho over
    [lo, hi] (clipped to [a, b]), integrated numerically in theta = acos(x),
    where d lambda rho = (1/pi) [g_0 mu_0 + 2 sum g_m mu_m cos(m theta)]
    d theta, by composite 8-point Gauss-Legendre quadrature with one panel
    per 1/(2M) of the theta range of a full period."""
    mu = np.asarray(mu, np.float64)
    M = mu.size
    g = kernel("jackson", M)[:M]
    xl = np.clip((2.0 * lo - a - b) / (b - a), -1.0, 1.0)
    xh = np.clip((2.0 * hi - a - b) / (b - a), -1.0, 1.0)
    t1, t2 = math.acos(xh), math.acos(xl)          # theta decreases with x
    if t2 <= t1:
        return 0.0
    npan = max(8, int(math.ceil(2 * M * (t2 - t1) / math.pi)))
    xg, wg = np.polynomial.legendre.leggauss(8)
    edges = np.linspace(t1, t2, npan + 1)
    h = 0.5 * (edges[1:] - edges[:-1])
    th = ((edges[:-1] + edges[1:]) * 0.5)[:, None] + h[:, None] * xg[None, :]
    w = h[:, None] * wg[None, :]
    m = np.arange(1, M)
    f = g[0] * mu[0] + 2.0 * (g[1:] * mu[1:] * np.cos(th[..., None] * m)).sum(-1)
    return float(D * (f * w).sum() / np.pi)


def dos_margin(mu, D, a, b, lo, hi, n_s, iters=60):
    """Eq. DOS:search: the smallest margin delta' >= 0 such that the search
    interval [lo - delta', hi + delta'] holds n_s states by the KPM count,
    found by bisection on [0, (b - a)/2] (returns (b - a)/2 when even that
    holds fewer)."""
    S = 0.5 * (b - a)
    if dos_count(mu, D, a, b, lo - S, hi + S) < n_s:
        return S
    l, r = 0.0, S
    for _ in range(iters):
        mid = 0.5 * (l + r)
        if dos_count(mu, D, a, b, lo - mid, hi + mid) >= n_s:
            r = mid
        else:
            l = mid
    return r


# closed-form models ----------------------------------------------------------
def effort_flat(ns_over_nt):
    """eta*N_S in units of eta_0 (S_w/delta) N_T for a flat DOS, Eq. (etanflat)."""
    r = np.asarray(ns_over_nt, np.float64)
    return 1.0 / (1.0 - 1.0 / r)


def effort_linear(ns_over_nt):
    """Same for a linear DOS, Eq. (etanlinear); minimal (=4) at N_S = 4 N_T."""
    r = np.asarray(ns_over_nt, np.float64)
    return np.sqrt(r) / (1.0 - np.sqrt(1.0 / r))


def intensity(n_b, nnzr, F_a, F_m, S_d, S_i):
    """Computational intensity I(n_b) of the augmented spMMVM (Sec. 4.2),
    in flop/byte."""
    num = nnzr * (F_a + F_m) + math.ceil(9 * F_a / 2) + math.ceil(11 * F_m / 2)
    return num / (nnzr / n_b * (S_d + S_i) + 5 * S_d)


# --------------------------------------------------------------------------
# the filter (Fig. fig:ChebFD) and dense pieces
# --------------------------------------------------------------------------
def filter_block(H: CSR, a, b, gam, X, moments=False):
    """Y = p(H) X following Fig. fig:ChebFD; optionally the 2 n_p + 1 moments
    per column (doubling reading), shape (2 n_p + 1, n_s)."""
    X = np.array(X, np.complex128, order="C", copy=True)
    gam = np.ascontiguousarray(gam, np.float64)
    n_p = gam.size - 1
    U = np.empty_like(X)
    W = np.empty_like(X)
    mom = np.empty((2 * n_p + 1, X.shape[1])) if moments else None
    rc = lib().orc_filter(H.n, *H.ptrs(), a, b, _p(gam), n_p, _p(X), _p(U), _p(W),
                          X.shape[1], _p(mom))
    if rc != 0:
        raise ValueError("orc_filter: n_p must be >= 2")
    return (X, mom) if moments else X


def moments_direct(H: CSR, a, b, X, n_mom):
    X = np.ascontiguousarray(X, np.complex128)
    mom = np.empty((n_mom, X.shape[1]))
    lib().orc_moments_direct(H.n, *H.ptrs(), a, b, _p(X), X.shape[1], n_mom, _p(mom))
    return mom


def gram_kahan(A, B):
    A = np.ascontiguousarray(A, np.complex128)
    B = np.ascontiguousarray(B, np.complex128)
    S = np.empty((A.shape[1], B.shape[1]), np.complex128)
    lib().orc_gram_kahan(A.shape[0], _p(A), A.shape[1], _p(B), B.shape[1], _p(S))
    return S


def jacobi_herm(A):
    A = np.array(A, np.complex128, order="C", copy=True)
    n = A.shape[0]
    w = np.empty(n)
    V = np.empty((n, n), np.complex128)
    lib().orc_jacobi_herm(n, _p(A), _p(w), _p(V))
    return w, V


def svqb(Y, tau=1e-12, seed=0, refill_offset=0):
    Y = np.array(Y, np.complex128, order="C", copy=True)
    T = np.empty_like(Y)
    nref = lib().orc_svqb(Y.shape[0], _p(Y), _p(T), Y.shape[1], tau, seed, refill_offset)
    return Y, nref


def rayleigh_ritz(H: CSR, Y):
    Y = np.array(Y, np.complex128, order="C", copy=True)
    W = np.empty_like(Y)
    T = np.empty_like(Y)
    ns = Y.shape[1]
    th = np.empty(ns)
    res = np.empty(ns)
    lib().orc_rayleigh_ritz(H.n, *H.ptrs(), _p(Y), _p(W), _p(T), ns, _p(th), _p(res))
    return th, Y, res


def harmonic_ritz(H: CSR, Y, tau):
    """Harmonic Ritz pairs of span(Y) (Y orthonormal) for the target tau:
    (rho ascending, unit vectors, residuals); see orc_harmonic_ritz."""
    Y = np.array(Y, np.complex128, order="C", copy=True)
    W = np.empty_like(Y)
    T = np.empty_like(Y)
    ns = Y.shape[1]
    rho = np.empty(ns)
    res = np.empty(ns)
    if lib().orc_harmonic_ritz(H.n, *H.ptrs(), _p(Y), _p(W), _p(T), ns, tau, _p(rho), _p(res)):
        raise ValueError("orc_harmonic_ritz: (H - tau) Y is rank deficient")
    return rho, Y, res


class _Stats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("n_found", C.c_int), ("n_mvm", C.c_int64),
                ("refilled", C.c_int), ("a", C.c_double), ("b", C.c_double)]


def chebfd_solve(H: CSR, lam_lo, lam_hi, n_s, n_p, kind="lanczos", mu=2.0, eps=1e-9,
                 max_iter=50, seed=1, a=float("nan"), b=float("nan"), vectors=True,
                 harmonic=False):
    """The ChebFD scheme of Sec. 3.1 (steps 1-8), optionally with harmonic
    Ritz extraction in step 7.  Returns (status, evals, residuals, evecs or
    None, stats dict)."""
    ev = np.empty(n_s)
    rs = np.empty(n_s)
    V = np.empty((H.n, n_s), np.complex128) if vectors else None
    st = _Stats()
    status = lib().orc_chebfd_solve(H.n, *H.ptrs(), lam_lo, lam_hi, n_s, n_p,
                                    KERNELS[kind] if isinstance(kind, str) else kind, mu, eps,
                                    max_iter, seed, a, b, _p(ev), _p(rs), _p(V), C.byref(st),
                                    1 if harmonic else 0)
    if status < 0:
        raise ValueError("orc_chebfd_solve: invalid arguments")
    f = st.n_found
    stats = dict(iterations=st.iterations, n_found=f, n_mvm=st.n_mvm, refilled=st.refilled,
                 a=st.a, b=st.b)
    return status, ev[:f].copy(), rs[:f].copy(), (V[:, :f].copy() if vectors else None), stats


def num_threads() -> int:
    return lib().orc_num_threads()
