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


N_MOM_COUNT = 4096   # moments for the eigenvalue count (resolution ~ pi S_w / M)


def kpm_count(mu, n, a, b, delta):
    """N_T = N sum_m g_m c_m mu_m for the window [-delta, delta] with the
    Jackson kernel (Eq. DOS:target)."""
    g = B.chebfd_coeffs(-delta, delta, a, b, len(mu) - 1, "jackson")
    return n * float(np.dot(g, mu))


def window_for_count(mu, n, a, b, n_target):
    """delta with N_T(delta) = n_target (bisection on the KPM count)."""
    lo, hi = 1e-6, 0.5 * (b - a)
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if kpm_count(mu, n, a, b, mid) < n_target:
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
    ap.add_argument("--polish-units", type=float, default=None,
                    help="complex64 forms: FP64 switch threshold in units of 2^-23 S_w "
                         "(default: the library's, 8 units)")
    ap.add_argument("--polish", default="correction", choices=["correction", "fp64"],
                    help="complex64 forms: FP32 correction passes or FP64 filter passes")
    ap.add_argument("--bounds", default="gershgorin", choices=["gershgorin", "lanczos"],
                    help="spectral interval: Gershgorin or 40 Lanczos steps (checked by the solver)")
    ap.add_argument("--plan-only", action="store_true",
                    help="only the window, the rule's N_p and the fused-step time per precision")
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
    lanczos_steps = 0
    if args.bounds == "lanczos":
        lanczos_steps = 40
        a, b = B.chebfd_lanczos_bounds(ctx, H, k=lanczos_steps, seed=w["seeds"][0])
    polish_switch = (float("nan") if args.polish_units is None
                     else args.polish_units * 2.0**-23 * max(abs(a), abs(b)))
    mu_c = B.chebfd_kpm_moments(ctx, H, learned.N_VEC, N_MOM_COUNT, w["seeds"][0], a, b,
                                precision=B.PREC_C64)
    mu = mu_c[:learned.N_MOM]
    delta = window_for_count(mu_c, n, a, b, w["n_target"])
    nt = kpm_count(mu_c, n, a, b, delta)
    # the rule's margin from the high-resolution moments: the search
    # interval must hold N_S eigenvalues, and 256 moments cannot resolve the
    # small margins of N_S/N_T near 1
    _, _, np_rule, margin = B.chebfd_dos_params(mu_c, n, a, b, -delta, delta, n_s=n_s,
                                                 ns_max=n_s, with_margin=True)
    print(json.dumps(dict(workload=args.workload, N=n, a=a, b=b, bounds=args.bounds, delta=delta,
                          nt_est=nt,
                          np_rule=np_rule, margin=margin,
                          setup_s=round(time.perf_counter() - t0, 2))), flush=True)
    if args.plan_only:
        import torch
        plan = dict(workload=args.workload, N=n, delta=delta, nt_est=nt, np_rule=np_rule)
        for name, prec, dt in (("c128", B.PREC_C128, torch.complex128),
                               ("c64", B.PREC_C64, torch.complex64)):
            X = torch.empty((n, n_s), dtype=dt, device="cuda")
            U, Wb = torch.empty_like(X), torch.empty_like(X)
            B.chebfd_random_block(ctx, X, seed=1)
            g = B.chebfd_coeffs(-delta, delta, a, b, 12)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            B.chebfd_filter_apply(ctx, H, g, a, b, X, U, Wb)
            torch.cuda.synchronize()
            step = (time.perf_counter() - t0) / 12
            plan[f"step_ms_{name}"] = round(step * 1e3, 2)
            plan[f"filter_pass_s_{name}"] = round(step * np_rule, 1)
            del X, U, Wb
            torch.cuda.empty_cache()
        print(json.dumps(plan), flush=True)
        with open(args.out, "w") as fh:
            json.dump(plan, fh, indent=1)
        return
    P = dict(H=H, n=n, a=a, b=b, delta=delta, mu=mu, mu_rule=mu_c,
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
                              max_iter=args.max_iter, seed=w["seeds"][0], verbose=1,
                              bounds=lanczos_steps, polish_switch=polish_switch,
                              polish=(B.POLISH_FP64 if args.polish == "fp64"
                                      else B.POLISH_CORRECTION))
        row = dict(form=form, n_p=n_p, corrections=corr is not None, status=r["rc"],
                   found=r["found"], time_s=r["time"], polish=args.polish,
                   n_mvm=r["n_mvm"], iterations=r["iterations"],
                   iterations_c64=r["iterations_c64"], iterations_corr=r["iterations_corr"],
                   history=r["history"],
                   max_residual=float(r["res"].max()) if r["found"] else None,
                   polish_units=args.polish_units)
        if form == "fp64":
            ref = r
        elif ref is not None and ref["found"] == r["found"] and r["found"]:
            S_w = max(abs(a), abs(b))
            row["max_eig_err_rel_Sw"] = float(np.abs(r["evals"] - ref["evals"]).max() / S_w)
            row["speedup_vs_fp64"] = ref["time"] / r["time"]
        print(json.dumps(row), flush=True)
        # eigenvalues in the file only, so runs made separately can be compared
        row["evals"] = [float(x) for x in r["evals"]]
        results[form] = row
        torch.cuda.empty_cache()
    out = dict(workload=args.workload, lattice=L, N=n, n_s=n_s, storage=args.storage,
               window=[-delta, delta], nt_est=nt, np_rule=np_rule, results=results)
    with open(args.out, "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
