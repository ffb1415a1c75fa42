"""CPU checks of the C-ABI library: it loads, exports every symbol the header
declares, validates arguments, and its host-side math (coefficients, filter
quality, parameter rule, small Hermitian eigensolver) agrees with the paper
and with the CPU reference.  No device computation happens here."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import chebfd_inputs as inp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def B():
    from paper_1510_04895_amd import binding
    binding.lib()
    return binding


def test_every_declared_symbol_is_exported(B):
    hdr = open(os.path.join(ROOT, "include", "chebfd.h")).read()
    declared = set(re.findall(r"\b(chebfd_[a-z_0-9]+)\s*\(", hdr))
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    assert declared, "no declarations found"
    assert declared <= exported, sorted(declared - exported)
    assert set(B.exported_symbols()) <= exported


def test_strerror_and_version(B):
    L = B.lib()
    assert L.chebfd_strerror(0) == b"ok"
    assert b"invalid" in L.chebfd_strerror(-1)
    assert L.chebfd_version().startswith(b"chebfd")


def test_create_without_device_fails_cleanly(B):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    h = C.c_void_p()
    rc = B.lib().chebfd_create(C.byref(h), 0, None)
    assert rc == -3 and not h
    assert B.lib().chebfd_last_error()


def test_coeffs_match_reference(B, orc):
    for (lo, hi, a, b, n_p, k) in [(-0.1, 0.1, -8.5, 8.5, 300, "lanczos"),
                                   (0.3, 0.9, -1.0, 2.0, 77, "jackson"),
                                   (-2.0, -1.5, -3.0, 3.0, 40, "fejer"),
                                   (-0.5, 0.5, -1.0, 1.0, 5, "none")]:
        g1 = B.chebfd_coeffs(lo, hi, a, b, n_p, k)
        g2 = orc.gamma(lo, hi, a, b, n_p, k)
        assert np.abs(g1 - g2).max() < 1e-13


@pytest.mark.parametrize("kind,n_p", [("lanczos", 120), ("jackson", 37), ("none", 2)])
def test_coeffs_divided_match_definition(B, orc, kind, n_p):
    """chebfd_coeffs_divided: q(y) = (p(y) - p(t)) / (y - t) for the filter
    polynomial p (evaluated by the reference, Clenshaw in the scaled
    variable) and the returned p(t), at points inside and outside the window
    and at the interval ends; q itself is summed here from its coefficients
    with T_n(y) = cos(n arccos y)."""
    a, b = -7.5, 8.25
    gam = orc.gamma(-0.4, 0.3, a, b, n_p, kind=kind)
    ys = np.linspace(-0.999, 0.999, 41)
    for lam in (-0.35, 0.0, 0.3, 1.7, -7.5, 8.25):
        d, pt = B.chebfd_coeffs_divided(gam, a, b, lam)
        assert d.shape == (n_p,)
        assert abs(pt - orc.poly_eval(gam, a, b, lam)) < 1e-13
        t = (2 * lam - a - b) / (b - a)
        for y in ys:
            if abs(y - t) < 1e-3:
                continue
            q = float(np.sum(d * np.cos(np.arange(n_p) * np.arccos(y))))
            x = 0.5 * ((b - a) * y + a + b)
            want = (orc.poly_eval(gam, a, b, x) - pt) / (y - t)
            assert abs(q - want) < 1e-11 * (1.0 + abs(want)), (lam, y, q, want)
    with pytest.raises(B.ChebFDError):
        B.chebfd_coeffs_divided(gam[:2], a, b, 0.0)


def test_coeffs_invalid_arguments(B):
    with pytest.raises(B.ChebFDError) as e:
        B.chebfd_coeffs(0.1, -0.1, -1, 1, 10)
    assert e.value.code == -1
    with pytest.raises(B.ChebFDError):
        B.chebfd_coeffs(-0.1, 0.1, -1, 1, 1)
    with pytest.raises(B.ChebFDError):
        B.chebfd_coeffs(2.0, 3.0, -1, 1, 10)          # window outside [a, b]
    with pytest.raises(B.ChebFDError):
        B.chebfd_coeffs(-0.1, 0.1, 1, -1, 10)


def test_filter_columns_rejects_bad_arguments_without_a_device(B):
    """chebfd_filter_apply_columns checks its arguments before any device
    call: NULL context, matrix or table -> INVALID_ARG; complex128 ->
    UNSUPPORTED (the per-column step exists for complex64 only)."""
    L = B.lib()
    dummy = C.c_void_p(8)
    assert L.chebfd_filter_apply_columns(None, dummy, B.PREC_C64, dummy, 4, 10, -1.0, 1.0,
                                         dummy, dummy, dummy, 4, 4) == -1
    assert L.chebfd_filter_apply_columns(dummy, None, B.PREC_C64, dummy, 4, 10, -1.0, 1.0,
                                         dummy, dummy, dummy, 4, 4) == -1
    assert L.chebfd_filter_apply_columns(dummy, dummy, B.PREC_C64, None, 4, 10, -1.0, 1.0,
                                         dummy, dummy, dummy, 4, 4) == -1
    assert L.chebfd_filter_apply_columns(dummy, dummy, B.PREC_C128, dummy, 4, 10, -1.0, 1.0,
                                         dummy, dummy, dummy, 4, 4) == -5
    assert b"complex64" in L.chebfd_last_error()


def test_filter_quality_matches_reference(B, orc):
    g = orc.gamma(-0.0025, 0.0025, -1, 1, 817)
    s1, e1 = B.chebfd_filter_quality(g, -1, 1, -0.0025, 0.0025, -0.01, 0.01)
    s2, e2 = orc.filter_quality(g, -1, 1, -0.0025, 0.0025, -0.01, 0.01)
    assert e1 == pytest.approx(e2, rel=2e-3)


@pytest.mark.parametrize("delta,ratio,np_pr", [(0.05, 1.0, 124), (0.05, 0.41, 303),
                                               (0.0025, 3.0, 817)])
def test_optimal_np_reproduces_table_num(B, delta, ratio, np_pr):
    """The library's own parameter rule reproduces Table tab:num."""
    dp = ratio * delta
    n, eta = B.chebfd_optimal_np(-1, 1, -delta, delta, -delta - dp, delta + dp)
    assert abs(n - np_pr) <= max(2, 0.025 * np_pr)


def test_host_eigh_vs_lapack(B):
    g = np.random.default_rng(0)
    for n in [1, 2, 3, 10, 64, 200]:
        M = g.normal(size=(n, n)) + 1j * g.normal(size=(n, n))
        A = M + M.conj().T
        w, V = B.chebfd_host_eigh(A)
        assert np.abs(w - np.linalg.eigvalsh(A)).max() < 1e-12 * max(1.0, np.abs(w).max())
        assert np.abs(A @ V - V * w).max() < 1e-11 * max(1.0, np.abs(w).max())
        assert np.abs(V.conj().T @ V - np.eye(n)).max() < 1e-12


def test_host_eigh_degenerate_and_diagonal(B, orc):
    # Kramers-degenerate TI spectrum and an already diagonal matrix
    H = orc.ti_hamiltonian(2, 2, 4, pbc=3, V=1.0, seed=4)
    A = H.dense()
    w, V = B.chebfd_host_eigh(A)
    assert np.abs(w - np.linalg.eigvalsh(A)).max() < 1e-12
    assert np.abs(A @ V - V * w).max() < 1e-12
    D = np.diag(np.array([3.0, -1.0, 2.0, 2.0, 0.5])).astype(complex)
    w, V = B.chebfd_host_eigh(D)
    assert np.allclose(w, [-1.0, 0.5, 2.0, 2.0, 3.0])
    with pytest.raises(B.ChebFDError):
        B.chebfd_host_eigh(np.full((3, 3), np.nan, complex))


def test_dos_params_count_and_rules(B, orc):
    """N_T from KPM moments (Eq. DOS:target) against the exact count of a
    small lattice; moments computed by the reference on random-phase
    vectors (stochastic trace), so the count is approximate."""
    H = orc.ti_hamiltonian(6, 6, 6, pbc=3, V=1.0, seed=2)
    a, b = orc.gershgorin(H)
    X = inp.random_phase_block(H.n, 24, seed=1)
    mu = orc.moments_direct(H, a, b, X, 256).mean(1) / H.n
    w = np.linalg.eigvalsh(H.dense())
    for d in (0.8, 1.5):
        exact = int((np.abs(w) <= d).sum())
        nt, ns, n_p = B.chebfd_dos_params(mu, H.n, a, b, -d, d, ns_over_nt=3.0)
        assert abs(nt - exact) <= 0.25 * exact + 4
        assert ns >= 16 and ns % 2 == 0 and ns >= 3 * nt - 2
        assert n_p > 8


def test_fit_corrections_lowers_sigma(B, orc):
    """The fitted hat amplitudes lower the damping factor sigma of Sec. 2.3,
    as evaluated independently by the reference on the corrected
    coefficients decoded by the library."""
    a, b, d = -1.0, 1.0, 0.02
    t_lo, t_hi, s_lo, s_hi = -d, d, -2 * d, 2 * d
    n_p = 300
    amp, sig_fit = B.chebfd_fit_corrections(a, b, t_lo, t_hi, s_lo, s_hi, n_p, iters=150)
    g0 = orc.gamma(t_lo, t_hi, a, b, n_p)
    s_plain, _ = orc.filter_quality(g0, a, b, t_lo, t_hi, s_lo, s_hi)
    out = np.concatenate([[0.0, 0.0], amp]).astype(np.float32)
    n_p2, ns, corr = B.chebfd_learned_decode(out, n_p, 64)
    assert n_p2 == n_p and ns == 64 and corr.size == n_p + 1
    s_corr, _ = orc.filter_quality(g0 * (1 + corr), a, b, t_lo, t_hi, s_lo, s_hi)
    assert s_corr < 0.9 * s_plain
    # a zero network output leaves the expansion unchanged
    n0, s0, c0 = B.chebfd_learned_decode(np.zeros(66, np.float32), 500, 40)
    assert n0 == 500 and s0 == 40 and np.all(c0 == 0.0)
    n1, s1, _ = B.chebfd_learned_decode(np.r_[np.log(2.0), -np.log(2.0), np.zeros(64)], 500, 40)
    assert n1 == 1000 and s1 == 20


def test_learned_features_layout(B):
    mu = np.linspace(1, 0, 10)
    f = B.chebfd_learned_features(mu, -4.0, 4.0, -0.4, 0.2)
    assert f.dtype == np.float32 and f.size == 12
    assert np.allclose(f[:10], mu) and np.allclose(f[10:], [-0.1, 0.05])


def test_missing_library_fails_loudly(tmp_path):
    """Without the built library every call raises (there is no CPU
    fallback): checked in a fresh interpreter with the library path pointed
    at a file that does not exist."""
    import subprocess
    import sys
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_1510_04895_amd import binding as B\n"
        "B.LIB_PATH = %r\n"
        "B._lib = None\n"
        "try:\n"
        "    B.chebfd_coeffs(-0.1, 0.1, -1.0, 1.0, 16)\n"
        "except RuntimeError as e:\n"
        "    print('raised:', e)\n"
        "    sys.exit(0)\n"
        "sys.exit(3)\n") % (ROOT, str(tmp_path / "libchebfd.so"))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "is missing" in r.stdout and "no CPU fallback" in r.stdout


def test_dos_params_match_oracle_density(B, orc):
    """The library's KPM count (Eq. DOS:target, a closed-form integral of the
    Jackson-damped expansion) and search margin (Eq. DOS:search, bisection)
    against the oracle's own density integrated by Gauss-Legendre
    quadrature and its own bisection, on the same moments."""
    H = orc.ti_hamiltonian(6, 6, 6, pbc=3, V=1.0, seed=2)
    a, b = orc.gershgorin(H)
    X = inp.random_phase_block(H.n, 24, seed=1)
    mu = orc.moments_direct(H, a, b, X, 256).mean(1) / H.n
    for d in (0.3, 0.8, 1.5):
        want = orc.dos_count(mu, H.n, a, b, -d, d)
        nt, ns, n_p = B.chebfd_dos_params(mu, H.n, a, b, -d, d, ns_over_nt=3.0)
        assert abs(nt - want) <= 1e-8 * max(1.0, want), (d, nt, want)
        nt2, ns2, n_p2, mg = B.chebfd_dos_params(mu, H.n, a, b, -d, d, n_s=120,
                                                 with_margin=True)
        mref = orc.dos_margin(mu, H.n, a, b, -d, d, 120)
        # the library floors the margin at the kernel width 2 S_w / M
        assert abs(mg - max(mref, (b - a) / 256)) <= 1e-9 * (b - a), (d, mg, mref)


def test_header_is_plain_c99(tmp_path):
    """include/chebfd.h is a C interface: it compiles as pedantic C99 with
    every warning an error, and a C caller can fill the parameter block."""
    src = tmp_path / "use_header.c"
    src.write_text('#include "chebfd.h"\n'
                   "int main(void) {\n"
                   "    chebfd_params p;\n"
                   "    chebfd_stats s;\n"
                   "    chebfd_iter_info h;\n"
                   "    (void)s; (void)h;\n"
                   "    return chebfd_params_default(&p) == 0 ? p.polish : 1;\n"
                   "}\n")
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
                        "-I" + os.path.join(ROOT, "include"), "-c", str(src), "-o",
                        str(tmp_path / "use_header.o")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
