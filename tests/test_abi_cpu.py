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
