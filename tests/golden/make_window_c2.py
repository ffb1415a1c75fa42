"""Writes the window spectrum of the 64x64x32 topological-insulator lattice
under tests/golden/, computed by the oracle's own ChebFD run.

The lattice is too large for dense diagonalisation (N = 524,288), so the
oracle runs the algorithm of Sec. 3.1 (steps 1-8) step by step: Gershgorin
bounds, the Lanczos-kernel window filter of Fig. fig:ChebFD on a CSR matrix,
SVQB with Kahan-compensated Gram sums, Rayleigh-Ritz with cyclic Jacobi,
residuals on the unscaled matrix, and the paper's exit rule.  Only
``oracle`` is called here.  The stored window is wider than the one the
tests use (|lambda| <= 0.2072) so that a test can check the gap around its
edges.

    python tests/golden/make_window_c2.py            # about 30-60 min on 8 cores
"""
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", ".."))
import oracle  # noqa: E402

L = (64, 64, 32)
SEED, V = 1, 1.0
DELTA = 0.23          # stored window half-width (the tests use 0.2072 inside it)
N_S, N_P = 256, 256   # search vectors and Lanczos-kernel degree
EPS = 1e-9


def main():
    t0 = time.time()
    H = oracle.ti_hamiltonian(*L, pbc=3, t=1.0, m=2.0, V=V, seed=SEED)
    a, b = oracle.gershgorin(H)
    print(f"matrix N={H.n} nnz={H.nnz} bounds [{a}, {b}] built in {time.time() - t0:.1f} s",
          flush=True)
    t0 = time.time()
    st, ev, rs, _, stats = oracle.chebfd_solve(H, -DELTA, DELTA, N_S, N_P, kind="lanczos",
                                               mu=2.0, eps=EPS, max_iter=30, seed=SEED,
                                               vectors=False)
    dt = time.time() - t0
    print(f"status {st}, {ev.size} pairs, max residual {rs.max():.3e}, "
          f"{stats['iterations']} iterations, {dt:.0f} s", flush=True)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                       f"ti_{L[0]}x{L[1]}x{L[2]}_V{V:g}_seed{SEED}_window{DELTA:g}.txt")
    hdr = (f"Eigenvalues in [-{DELTA}, {DELTA}] of Eq. (Ham), Sec. 5.1: lattice "
           f"{L[0]}x{L[1]}x{L[2]} (periodic x,y; open z), t=1, m=2, V={V:g}, disorder seed "
           f"{SEED}; N={H.n}.\n"
           f"Computed by oracle.chebfd_solve (Sec. 3.1 steps 1-8, FP64, CSR): N_S={N_S}, "
           f"N_p={N_P}, Lanczos kernel mu=2, eps={EPS:g}, Gershgorin [{a:.6f}, {b:.6f}], "
           f"status {st}, {stats['iterations']} iterations, {oracle.num_threads()} threads, "
           f"{dt:.0f} s.\n"
           f"Columns: eigenvalue, residual ||Hv - lambda v||.\n"
           f"Written by: python tests/golden/make_window_c2.py")
    np.savetxt(out, np.c_[ev, rs], fmt="%.17e", header=hdr)
    print(out, flush=True)


if __name__ == "__main__":
    main()
