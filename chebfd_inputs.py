"""Seeded synthetic inputs shared by the tests, the benchmark and smoke().

This module holds no arithmetic of the method: only workload definitions and
seeded random data (blocks, coefficient sequences, sparse test matrices,
diagonal spectra).  Both the oracle-side and the GPU-side tests take their
inputs from here.  The paper's own workloads are generated matrices (Sec. 5.1
and 5.4); the definitions below restate them at one-GPU sizes.
"""
from __future__ import annotations

import numpy as np

# --------------------------------------------------------------------------
# Topological-insulator lattices (Sec. 5.1, Eq. (Ham)): periodic x,y (pbc=3),
# open z, t=1, m=2, box disorder of width V.
# --------------------------------------------------------------------------
WORKLOADS = {
    # correctness configuration: dense spectrum known, 16 eigenvalues in window
    "ti_8x8x8": dict(L=(8, 8, 8), pbc=3, V=1.0, seeds=(1, 2, 3), n_s=32, n_p=200,
                     kernel="lanczos", mu=2.0, eps=1e-9, n_target=16),
    # the FP64 throughput configuration
    "ti_64x64x32": dict(L=(64, 64, 32), pbc=3, V=1.0, seeds=(1,), n_s=256, kernel="lanczos",
                        mu=2.0, eps=1e-9, n_target=64, delta=0.2072, sell_C=32, sell_sigma=256),
    # precision form
    "ti_128x128x64": dict(L=(128, 128, 64), pbc=3, V=1.0, seeds=(1,), n_s=256,
                          kernel="lanczos", mu=2.0, eps=1e-9, n_target=100, delta=0.1335),
    # learned form: disorder strength per realisation W ~ U[0,2]
    "ti_32x32x16": dict(L=(32, 32, 16), pbc=3, train_seeds=tuple(range(1, 201)),
                        heldout_seeds=tuple(range(10001, 10021)), n_kpm_vec=8, n_kpm_mom=256),
    # largest single-GPU lattice
    "ti_256x256x64": dict(L=(256, 256, 64), pbc=3, V=1.0, seeds=(1,), n_s=128,
                          kernel="lanczos", mu=2.0, eps=1e-9, n_target=100),
}


def ti_dim(L) -> int:
    return 4 * L[0] * L[1] * L[2]


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def random_block(n: int, n_s: int, seed: int, dtype=np.complex128) -> np.ndarray:
    """Complex block with entries uniform in the unit square [-1,1]^2."""
    g = rng(seed)
    X = g.uniform(-1, 1, (n, n_s)) + 1j * g.uniform(-1, 1, (n, n_s))
    return X.astype(dtype)


def random_gamma(n_p: int, seed: int) -> np.ndarray:
    """Arbitrary coefficient sequence gamma_0..gamma_{n_p} (the filter is
    linear in the coefficients, so any sequence exercises it)."""
    return rng(seed).uniform(-1, 1, n_p + 1) / np.sqrt(n_p + 1)


def random_phase_block(n: int, n_vec: int, seed: int) -> np.ndarray:
    """Unit-modulus random-phase vectors e^{2 pi i u} (stochastic trace)."""
    u = rng(seed).uniform(0, 1, (n, n_vec))
    return np.exp(2j * np.pi * u)


def flat_spectrum(D: int) -> np.ndarray:
    """Equidistant eigenvalues -1 + 2i/(D+1), i=1..D (Sec. 2.2)."""
    return -1.0 + 2.0 * np.arange(1, D + 1) / (D + 1)


def linear_spectrum(D: int) -> np.ndarray:
    """D eigenvalues in [-1,1] with density proportional to |lambda|: the k-th
    positive one is sqrt((k - 1/2)/(D/2)), mirrored to negative values."""
    k = np.arange(1, D // 2 + 1)
    pos = np.sqrt((k - 0.5) / (D / 2))
    return np.sort(np.concatenate([-pos, pos]))


def random_hermitian_csr(n: int, seed: int, min_row=1, max_row=24, diag_shift=0.0):
    """Random sparse Hermitian matrix with ragged row lengths (CSR: int64
    rowptr, int32 col, complex128 val, columns sorted, no duplicates)."""
    g = rng(seed)
    rows = {i: {} for i in range(n)}
    for i in range(n):
        rows[i][i] = complex(g.uniform(-1, 1) + diag_shift, 0.0)
        k = int(g.integers(min_row, max_row + 1)) // 2
        for j in g.integers(0, n, k):
            j = int(j)
            if j == i:
                continue
            v = complex(g.uniform(-1, 1), g.uniform(-1, 1)) * 0.5
            rows[i][j] = v
            rows[j][i] = v.conjugate()
    rowptr = np.zeros(n + 1, np.int64)
    cols, vals = [], []
    for i in range(n):
        cs = sorted(rows[i])
        cols.extend(cs)
        vals.extend(rows[i][c] for c in cs)
        rowptr[i + 1] = len(cols)
    return rowptr, np.array(cols, np.int32), np.array(vals, np.complex128)


def learned_sample(seed: int):
    """Disorder strength W ~ U[0, 2] and relative window half-width
    delta / S_w log-uniform in [1e-3, 5e-2] for one realisation of the
    learned-form workload (32x32x16 lattice)."""
    g = rng(1_000_003 * seed + 17)
    W = float(g.uniform(0.0, 2.0))
    rel = float(10 ** g.uniform(np.log10(1e-3), np.log10(5e-2)))
    return W, rel
