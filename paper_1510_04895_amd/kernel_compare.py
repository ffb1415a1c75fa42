"""Damping kernels compared at one lattice (Sec. 2.1, Table tab:Kernel;
the comparison of Sec. 5.2 / Fig. fig:ConvTopi).

    python -m paper_1510_04895_amd.kernel_compare WORKLOAD OUT.json [--storage sell]

For the workload's lattice and window (half-width `delta` of the workload
table, Gershgorin bounds, N_S of the workload): the plain FP64 solve with
the Lanczos kernel (mu = 1, 2, 3) and the Jackson kernel, each at its own
eta-minimising degree for the search margin delta' = delta (sqrt(N_S/N_T)
- 1) (Sec. 2.3-2.4), and all of them at the Lanczos mu = 2 degree, which
isolates the kernel.  Each run reports iterations, matrix-vector products,
time, and whether its eigenvalues equal the reference window stored under
tests/golden (when one exists for the workload).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

KERNEL_CASES = (("lanczos", 1.0), ("lanczos", 2.0), ("lanczos", 3.0), ("jackson", 0.0))
GOLDEN = {"ti_64x64x32": "ti_64x64x32_V1_seed1_window0.23.txt"}


def main():
    import torch
    import chebfd_inputs as inp
    ap = argparse.ArgumentParser()
    ap.add_argument("workload")
    ap.add_argument("out")
    ap.add_argument("--storage", default="sell", choices=["sell", "stencil"])
    args = ap.parse_args()
    w = inp.WORKLOADS[args.workload]
    ctx = B.Context(0)
    st = B.STORAGE_SELL if args.storage == "sell" else B.STORAGE_STENCIL
    H = B.Matrix.ti(ctx, w["L"], pbc=w["pbc"], V=w["V"], seed=w["seeds"][0], storage=st,
                    sell_C=w.get("sell_C", 32), sell_sigma=w.get("sell_sigma", 256))
    info = H.info()
    a, b = info["g_lo"], info["g_hi"]
    S_w = max(abs(a), abs(b))
    d, n_s = w["delta"], w["n_s"]
    dp = d * (math.sqrt(n_s / w["n_target"]) - 1.0)
    ref = None
    if args.workload in GOLDEN:
        g = np.sort(np.loadtxt(os.path.join(ROOT, "tests", "golden", GOLDEN[args.workload]))[:, 0])
        ref = g[np.abs(g) <= d]
    np_ref = B.chebfd_optimal_np(a, b, -d, d, -d - dp, d + dp, kernel="lanczos", mu=2.0)[0]
    runs = []
    for kern, mu in KERNEL_CASES:
        np_own, eta = B.chebfd_optimal_np(a, b, -d, d, -d - dp, d + dp, kernel=kern, mu=mu)
        for tag, n_p in (("own degree", np_own), ("lanczos mu=2 degree", np_ref)):
            p = B.default_params(lam_lo=-d, lam_hi=d, n_s=n_s, n_p=int(n_p), kernel=kern, mu=mu,
                                 eps=w["eps"], max_iter=60, lock=1, seed=w["seeds"][0],
                                 vectors=0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, ev, rs, _, stats = B.chebfd_solve(ctx, H, p)
            torch.cuda.synchronize()
            T = time.perf_counter() - t0
            r = dict(kernel=kern, mu=mu if kern == "lanczos" else None, degree=tag,
                     n_p=int(n_p), eta=float(eta) if tag == "own degree" else None,
                     status=int(rc), found=int(ev.size), iterations=stats["iterations"],
                     n_mvm=int(stats["n_mvm"]), time_s=round(T, 3),
                     max_residual=float(rs.max()) if rs.size else None)
            if ref is not None:
                r["matches_oracle_window"] = bool(ev.size == ref.size and
                                                  np.abs(ev - ref).max() < 1e-10 * S_w)
            runs.append(r)
            print(json.dumps(r), flush=True)
    out = dict(workload=args.workload, storage=args.storage, bounds=[a, b], window=[-d, d],
               n_s=n_s, margin=dp, runs=runs)
    with open(args.out, "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
