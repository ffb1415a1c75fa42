"""The paper's topological-insulator experiment at one-GPU scale (Sec. 5.2,
Fig. fig:ConvTopi and Fig. fig:EffortTopi).

    python -m paper_1510_04895_amd.ti_experiment OUT.json [--part grid,kernels]
        [--cases NS:NP:KERNEL:MU,...]

Eq. (Ham) on a 256 x 256 x 10 slab (periodic x, y; open z; D = 2,621,440),
t = 1, disorder V_n uniform in [-1, 1] (V = 2), spectral interval fixed at
[a, b] = [-5.5, 5.5], target interval I_T = [-0.06, 0.06], residual goal
1e-9, FP64 throughout (complex128, matrix-free).  As in the paper no pair is
locked, so every iteration filters all N_S search vectors and the effort is
N_MVM = N_p x N_S x iterations.

  grid:    N_S in {224, 256, 304} x N_p in {862, 1438, 2590}, Lanczos kernel
           mu = 2 (the nine points where the two panels of Fig.
           fig:EffortTopi cross);
  kernels: N_S = 256, N_p = 1438 with the Jackson kernel and the Lanczos
           kernel for mu = 1, 2, 3, with the residual history of Fig.
           fig:ConvTopi (smallest in-window residual, largest accepted one,
           against N_MVM).

The disorder realisation here is seed 1 of the generator, so N_T differs
from the paper's 144; the KPM estimate of Eq. DOS:target (2048 moments of 16
random-phase vectors) is reported beside the converged count, and the
linear-DOS effort estimate of Eq. (etanlinear) -- eta_opt(delta') N_S
(-log10 eps) with delta' = delta (sqrt(N_S/N_T) - 1), minimised over N_S --
is evaluated for the converged N_T.  Every run must find the same
eigenvalues (count and values to 1e-10 S_w).
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from . import binding as B
from . import scale_runs

L = (256, 256, 10)
V = 2.0
A, BB = -5.5, 5.5
DELTA = 0.06
EPS = 1e-9
GRID_NS = (224, 256, 304)
GRID_NP = (862, 1438, 2590)
KERNEL_CASES = (("jackson", 2.0), ("lanczos", 1.0), ("lanczos", 2.0), ("lanczos", 3.0))
PAPER = {"n_t": 144, "n_t_dos_estimate": 124, "best_n_mvm": 1.2e6, "theory_min_n_mvm": 1.06e6}


def solve(ctx, H, n_s, n_p, kernel, mu, seed=1, max_iter=40):
    p = B.default_params(lam_lo=-DELTA, lam_hi=DELTA, n_s=n_s, n_p=n_p, kernel=kernel, mu=mu,
                         eps=EPS, max_iter=max_iter, lock=0, a=A, b=BB, seed=seed, vectors=0)
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, ev, rs, _, st = B.chebfd_solve(ctx, H, p)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    return dict(n_s=n_s, n_p=n_p, kernel=kernel, mu=mu, status=int(rc), time_s=round(T, 2),
                iterations=st["iterations"], n_mvm=int(st["iterations"] * n_s * n_p),
                n_found=int(ev.size), max_residual=float(rs.max()) if rs.size else None,
                history=[{k: h[k] for k in ("n_mvm", "n_window", "n_accepted", "n_converged",
                                            "n_locked", "r_min", "r_max_accepted")}
                         for h in st["history"]]), ev


def theory_min(n_t):
    """Linear-DOS estimate of the minimal effort (Eq. etanlinear with the
    eta-minimising degree for each N_S; Sec. 2.3-2.4)."""
    best = None
    for n_s in range(max(n_t + 2, 16), 8 * n_t, 4):
        dp = DELTA * (math.sqrt(n_s / n_t) - 1.0)
        n_p, eta = B.chebfd_optimal_np(A, BB, -DELTA, DELTA, -DELTA - dp, DELTA + dp)
        mvm = eta * (-math.log10(EPS)) * n_s
        if best is None or mvm < best["n_mvm"]:
            best = dict(n_mvm=mvm, n_s=n_s, n_p=n_p, delta_margin=dp)
    return best


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("out")
    ap.add_argument("--part", default="grid,kernels")
    ap.add_argument("--cases", default="",
                    help="explicit runs NS:NP:KERNEL:MU (comma separated) instead of --part")
    args = ap.parse_args()
    ctx = B.Context(0)
    H = B.Matrix.ti(ctx, L, pbc=3, V=V, seed=1, storage=B.STORAGE_STENCIL)
    info = H.info()
    n = info["n"]
    lo, hi = B.chebfd_lanczos_bounds(ctx, H, k=60, seed=1, pad=0.0)
    mu_k = B.chebfd_kpm_moments(ctx, H, 16, 2048, 7, A, BB, precision=B.PREC_C128)
    nt_kpm = scale_runs.kpm_count(mu_k, n, A, BB, DELTA)
    out = dict(lattice="x".join(map(str, L)), D=n, V=V, interval=[A, BB], window=[-DELTA, DELTA],
               eps=EPS, lanczos_extremes=[lo, hi], n_t_kpm_estimate=round(nt_kpm, 1),
               paper=PAPER, runs=[])
    print(f"# D={n}, Lanczos extremes [{lo:.4f}, {hi:.4f}], KPM N_T estimate {nt_kpm:.1f}",
          flush=True)
    if not (A < lo and hi < BB):
        raise SystemExit("the spectrum leaves [-5.5, 5.5]; the fixed interval of Sec. 5.2 "
                         "does not hold for this realisation")
    ref = None
    S_w = max(abs(A), abs(BB))
    parts = args.part.split(",") if not args.cases else []
    cases = []
    for c in filter(None, args.cases.split(",")):
        ns, npp, k, m = c.split(":")
        cases.append((int(ns), int(npp), k, float(m), "cases"))
    if "grid" in parts:
        cases += [(ns, npp, "lanczos", 2.0, "grid") for ns in GRID_NS for npp in GRID_NP]
    if "kernels" in parts:
        cases += [(256, 1438, k, m, "kernels") for k, m in KERNEL_CASES
                  if not ("grid" in parts and k == "lanczos" and m == 2.0)]
    for ns, npp, k, m, tag in cases:
        r, ev = solve(ctx, H, ns, npp, k, m)
        r["part"] = tag
        if ref is None and r["status"] == 0:
            ref = ev
        # effort until every window pair had converged (the paper stops
        # there; the exit rule runs one confirming iteration more)
        full = [h["n_mvm"] for h in r["history"] if ref is not None and
                h["n_converged"] + h["n_locked"] >= ref.size]
        r["n_mvm_all_converged"] = int(full[0]) if full else None
        r["same_eigenvalues"] = bool(ref is not None and ev.size == ref.size and
                                     (ev.size == 0 or np.abs(ev - ref).max() < 1e-10 * S_w))
        out["runs"].append(r)
        print(f"# N_S {ns} N_p {npp} {k} mu {m}: status {r['status']}, {r['iterations']} "
              f"iterations, N_MVM {r['n_mvm']:.3e}, {r['n_found']} pairs, "
              f"{r['time_s']} s, same {r['same_eigenvalues']}", flush=True)
        with open(args.out, "w") as fh:
            json.dump(out, fh, indent=1)
    if ref is not None:
        out["n_t"] = int(ref.size)
        out["theory_min"] = theory_min(int(ref.size))
        ok = [r for r in out["runs"] if r["status"] == 0 and r["same_eigenvalues"]]
        if ok:
            best = min(ok, key=lambda r: r["n_mvm_all_converged"] or r["n_mvm"])
            out["best"] = {k: best[k] for k in ("n_s", "n_p", "kernel", "mu", "n_mvm",
                                                "n_mvm_all_converged", "iterations")}
        out["eigenvalues"] = [float(v) for v in ref]
    with open(args.out, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps({k: out.get(k) for k in ("n_t", "n_t_kpm_estimate", "best", "theory_min")}),
          flush=True)


if __name__ == "__main__":
    main()
