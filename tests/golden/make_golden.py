"""Writes the dense-spectrum fixtures under tests/golden/.

Each fixture is the full spectrum of the topological-insulator Hamiltonian of
Sec. 5.1, Eq. (Ham) (periodic x,y, open z, t=1, m=2, box disorder of width
V from the stated seed), computed by the oracle's own cyclic Jacobi
diagonalisation.  Only ``oracle`` is called here.

    python tests/golden/make_golden.py 8 8 8 1      # Lx Ly Lz seed
"""
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", ".."))
import oracle  # noqa: E402


def main(Lx, Ly, Lz, seed, V=1.0):
    H = oracle.ti_hamiltonian(Lx, Ly, Lz, pbc=3, t=1.0, m=2.0, V=V, seed=seed)
    t0 = time.time()
    w, _ = oracle.jacobi_herm(H.dense())
    dt = time.time() - t0
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                       f"ti_{Lx}x{Ly}x{Lz}_V{V:g}_seed{seed}_evals.txt")
    hdr = (f"Full spectrum of Eq. (Ham), Sec. 5.1: lattice {Lx}x{Ly}x{Lz} (periodic x,y; open z), "
           f"t=1, m=2, V={V:g}, disorder seed {seed}; N={H.n}.\n"
           f"Computed by oracle.jacobi_herm (cyclic Jacobi, FP64) in {dt:.0f} s.\n"
           f"Written by: python tests/golden/make_golden.py {Lx} {Ly} {Lz} {seed}")
    np.savetxt(out, w, fmt="%.17e", header=hdr)
    print(out, dt)


if __name__ == "__main__":
    a = [int(x) for x in sys.argv[1:5]]
    main(*a)
