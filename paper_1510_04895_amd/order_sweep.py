"""Times the fused filter step under each block order on the TI lattices of
the throughput, precision and largest configurations, both storages and
both precisions, one JSON line per case.

    python -m paper_1510_04895_amd.order_sweep [stencil,sell]

Each case is the average of 20 (10 at 256x256x64) fused MODE_STEP launches
timed with HIP events on the library stream; GB/s counts the five block
streams (u read, w read and written, x read and written) only.
"""
from __future__ import annotations

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CASES = [("ti_64x64x32", 20), ("ti_128x128x64", 20), ("ti_256x256x64", 10)]


def main(argv):
    sys.path.insert(0, ROOT)
    import torch
    import bench
    import chebfd_inputs as inp
    from paper_1510_04895_amd import binding as B

    storages = argv[0].split(",") if argv else ["stencil", "sell"]
    ctx = B.Context(0)
    for name, steps in CASES:
        w = inp.WORKLOADS[name]
        L, n_s = w["L"], w["n_s"]
        for st in storages:
            if st == "sell" and L[0] >= 256:
                continue   # the largest lattice runs matrix-free only
            t0 = time.time()
            H = B.Matrix.ti(ctx, L, pbc=w["pbc"], V=w["V"], seed=w["seeds"][0],
                            storage=B.STORAGE_SELL if st == "sell" else B.STORAGE_STENCIL)
            print(f"# built {name} {st} in {time.time() - t0:.1f} s", flush=True)
            for prec in (B.PREC_C128, B.PREC_C64):
                s_d = 16 if prec == B.PREC_C128 else 8
                vec_bytes = 5 * H.info()["n"] * n_s * s_d
                for order in (0, 2):
                    B.chebfd_set_tuning(ctx, "order", order)
                    t = bench.time_fused(B, ctx, H, prec, n_s, 0.1, steps)
                    print(json.dumps(dict(workload=name, storage=st,
                                          prec="c128" if prec == B.PREC_C128 else "c64",
                                          order=order, ms=round(t * 1e3, 3),
                                          vec_GBs=round(vec_bytes / t / 1e9, 1))), flush=True)
            B.chebfd_set_tuning(ctx, "order", -1)
            del H
            torch.cuda.synchronize()


if __name__ == "__main__":
    main(sys.argv[1:])
