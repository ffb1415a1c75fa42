"""Precision-form and learned-form runs at the larger lattices.

    python -m paper_1510_04895_amd.scale_runs WORKLOAD OUT.json [--storage stencil]
                                             [--forms fp64,c64,c64_learned]

For the workload's lattice: the window [-delta, delta] is chosen from the KPM
density of states so that it holds about n_target eigenvalues (Eq.
DOS:target); then the plain FP64 solve, the complex64 sweep with FP64
orthogonalisation / Rayleigh-Ritz / polish, and (optionally) the complex64
sweep with the learned filter degree and coefficient corrections are run to
residual eps, and the eigenvalue / residual errors of the complex64 forms
against the FP64 run are reported.
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
from . import learned

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def window_for_count(mu, n, a, b, n_target, n_s):
    """delta with N_T(delta) = n_target from the KPM estimate (bisection)."""
    lo, hi = 1e-6, 0.5 * (b - a)
    for _ in range(50):
        mid = 0.5 * (lo + hi)
        nt = B.chebfd_dos_params(mu, n, a, b, -mid, mid, n_s=n_s, ns_max=max(n_s, 2))[0]
        if nt < n_target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def main():
    import torch
    import chebfd_inputs as inp
    ap = argparse.ArgumentParser()
    ap.add_argument("workload")
    ap.add_argument("out")
    ap.add_argument("--storage", default="stencil", choices=["sell", "stencil"])
    ap.add_argument("--forms", default="fp64,c64,c64_learned")
    ap.add_argument("--max-iter", type=int, default=40)
    ap.add_argument("--model", default=os.path.join(ROOT, "paper_1510_04895_amd", "models",
                                                     "ti_32x32x16_mlp.npz"))
    args = ap.parse_args()
    w = inp.WORKLOADS[args.workload]
    L, n_s = w["L"], w["n_s"]
    ctx = B.Context(0)
    st = B.STORAGE_SELL if args.storage == "sell" else B.STORAGE_STENCIL
    t0 = time.perf_counter()
    H = B.Matrix.ti(ctx, L, pbc=w["pbc"], V=w["V"], seed=w["seeds"][0], storage=st)
    info = H.info()
    n, a, b = info["n"], info["g_lo"], info["g_hi"]
    mu = B.chebfd_kpm_moments(ctx, H, learned.N_VEC, learned.N_MOM, w["seeds"][0], a, b,
                              precision=B.PREC_C64)
    delta = window_for_count(mu, n, a, b, w["n_target"], n_s)
    nt, _, np_rule, margin = B.chebfd_dos_params(mu, n, a, b, -delta, delta, n_s=n_s,
                                                  ns_max=n_s, with_margin=True)
    print(json.dumps(dict(workload=args.workload, N=n, a=a, b=b, delta=delta, nt_est=nt,
                          np_rule=np_rule, margin=margin,
                          setup_s=round(time.perf_counter() - t0, 2))), flush=True)
    P = dict(H=H, n=n, a=a, b=b, delta=delta, mu=mu,
             feats=B.chebfd_learned_features(mu, a, b, -delta, delta), nt=nt, ns0=n_s,
             np0=np_rule)
    results = {}
    ref = None
    for form in args.forms.split(","):
        corr, n_p = None, np_rule
        prec = B.PREC_C128 if form == "fp64" else B.PREC_C64
        if form == "c64_learned":
            net = learned.load_model(ctx, args.model)
            n_p, _, corr = learned.predict(ctx, net, P, n_s_fixed=n_s)
        torch.cuda.synchronize()
        r = learned.run_solve(ctx, H, delta, n_s, n_p, corr=corr, precision=prec,
                              max_iter=args.max_iter, seed=w["seeds"][0])
        row = dict(form=form, n_p=n_p, status=r["rc"], found=r["found"], time_s=r["time"],
                   n_mvm=r["n_mvm"], iterations=r["iterations"],
                   max_residual=float(r["res"].max()) if r["found"] else None)
        if form == "fp64":
            ref = r
        elif ref is not None and ref["found"] == r["found"] and r["found"]:
            S_w = max(abs(a), abs(b))
            row["max_eig_err_rel_Sw"] = float(np.abs(r["evals"] - ref["evals"]).max() / S_w)
            row["speedup_vs_fp64"] = ref["time"] / r["time"]
        results[form] = row
        print(json.dumps(row), flush=True)
        torch.cuda.empty_cache()
    out = dict(workload=args.workload, lattice=L, N=n, n_s=n_s, storage=args.storage,
               window=[-delta, delta], nt_est=nt, np_rule=np_rule, results=results)
    with open(args.out, "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
