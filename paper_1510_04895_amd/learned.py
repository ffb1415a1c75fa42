"""The learned form: a small network maps stochastic KPM moments of the
density of states plus the target window to the filter degree, the number of
search vectors (as ratios to the rule-based choice) and 64 hat amplitudes of
multiplicative coefficient corrections.  Training data come from runs of the
plain method itself; the network is trained on the GPU with the library's
own forward/backward/Adam kernels.  The rule-based choice
(chebfd_dos_params) is the fallback: a zero network output reproduces it.

    python -m paper_1510_04895_amd.learned sweep  OUT.npz SEED0 SEED1
    python -m paper_1510_04895_amd.learned fit    OUT.npz IN.npz [IN.npz ...]
    python -m paper_1510_04895_amd.learned train  MODEL.npz DATA.npz
    python -m paper_1510_04895_amd.learned eval   RESULT.json MODEL.npz SEED0 SEED1
"""
from __future__ import annotations

import json
import math
import os
import sys
import time

import numpy as np

from . import binding as B

L_DEFAULT = (32, 32, 16)
N_VEC, N_MOM = 8, 256
N_HAT, C_MAX = 64, 0.5
HIDDEN = 256
NS_MAX = 256


def _inputs():
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import chebfd_inputs
    return chebfd_inputs


def problem(ctx, seed, L=L_DEFAULT, storage=B.STORAGE_STENCIL):
    """Matrix, spectral interval, window and KPM features of one realisation."""
    W, rel = _inputs().learned_sample(seed)
    H = B.Matrix.ti(ctx, L, pbc=3, V=W, seed=seed, storage=storage)
    info = H.info()
    a, b = info["g_lo"], info["g_hi"]
    S_w = max(abs(a), abs(b))
    delta = rel * S_w
    mu = B.chebfd_kpm_moments(ctx, H, N_VEC, N_MOM, seed, a, b, precision=B.PREC_C64)
    feats = B.chebfd_learned_features(mu, a, b, -delta, delta)
    nt, ns0, np0 = B.chebfd_dos_params(mu, info["n"], a, b, -delta, delta, 3.0, ns_max=NS_MAX)
    return dict(H=H, n=info["n"], a=a, b=b, W=W, delta=delta, mu=mu, feats=feats, nt=nt,
                ns0=ns0, np0=np0)


def run_solve(ctx, H, delta, n_s, n_p, corr=None, precision=B.PREC_C128, max_iter=40, seed=1,
              verbose=0, bounds=0, polish_switch=float("nan"), polish=B.POLISH_CORRECTION):
    p = B.default_params(lam_lo=-delta, lam_hi=delta, n_s=n_s, n_p=n_p, eps=1e-9,
                         max_iter=max_iter, precision=precision, lock=1, seed=seed, vectors=0,
                         gamma_corr=corr, verbose=verbose, bounds=bounds,
                         polish_switch=polish_switch, polish=polish)
    t0 = time.perf_counter()
    rc, ev, rs, _, st = B.chebfd_solve(ctx, H, p)
    dt = time.perf_counter() - t0
    return dict(rc=int(rc), time=dt, found=int(len(ev)), evals=ev, res=rs, n_mvm=st["n_mvm"],
                iterations=st["iterations"], iterations_c64=st["iterations_c64"],
                iterations_corr=st["iterations_corr"],
                history=[(h["precision"], h["n_mvm"]) for h in st["history"]])


# sweep grid around the rule (N_S = 3 N_T, eta-optimal N_p): search spaces
# from about 1.35 N_T (the largest lattice's ratio) to 4.5 N_T, degrees from
# 0.6 to 1.6 times the rule's
NS_FACTORS = (0.45, 0.7, 1.0, 1.5)
NP_FACTORS = (0.6, 0.8, 1.0, 1.25, 1.6)


def sweep(out_path, seeds):
    """Plain-method sweep around the rule-based (N_S, N_p) for each seed; the
    label is the point with the fewest matrix-vector products (a count that
    does not depend on the machine) among those that find every pair."""
    import torch
    ctx = B.Context(0)
    recs = []
    for s in seeds:
        P = problem(ctx, s)
        ns0, np0 = P["ns0"], P["np0"]
        cand = []
        for fs in NS_FACTORS:
            ns = int(min(NS_MAX, max(16, round(ns0 * fs / 2) * 2)))
            for fp in NP_FACTORS:
                cand.append((ns, max(8, int(round(np0 * fp)))))
        cand = sorted(set(cand) | {(ns0, np0)})
        runs = [(ns, npp, run_solve(ctx, P["H"], P["delta"], ns, npp, seed=s)) for ns, npp in cand]
        top = max(r["found"] for _, _, r in runs)
        ok = [(r["n_mvm"], r["time"], ns, npp) for ns, npp, r in runs
              if r["rc"] == 0 and r["found"] == top]
        best = (min(ok) if ok else min((r["n_mvm"], r["time"], ns, npp) for ns, npp, r in runs))[1:]
        margin = B.chebfd_dos_params(P["mu"], P["n"], P["a"], P["b"], -P["delta"], P["delta"],
                                     n_s=best[1], ns_max=NS_MAX, with_margin=True)[3]
        recs.append(dict(seed=s, W=P["W"], delta=P["delta"], a=P["a"], b=P["b"], n=P["n"],
                         feats=P["feats"], nt=P["nt"], ns0=ns0, np0=np0, best_ns=best[1],
                         best_np=best[2], best_time=best[0], found=top, margin=margin,
                         mvm_best=int(min(ok)[0]) if ok else -1,
                         runs=[(ns, npp, r["time"], r["found"], r["rc"], int(r["n_mvm"]))
                               for ns, npp, r in runs]))
        print(json.dumps(dict(seed=s, W=round(P["W"], 3), delta=round(P["delta"], 5),
                              nt=round(P["nt"], 1), found=top, ns0=ns0, np0=np0,
                              best=best[1:], t_best=round(best[0], 3),
                              t_rule=round([r["time"] for ns, npp, r in runs
                                            if ns == ns0 and npp == np0][0], 3))), flush=True)
        _save_sweep(out_path, recs)
        torch.cuda.empty_cache()
    return recs


def _save_sweep(path, recs):
    np.savez(path, seed=np.array([r["seed"] for r in recs]),
             W=np.array([r["W"] for r in recs]), delta=np.array([r["delta"] for r in recs]),
             a=np.array([r["a"] for r in recs]), b=np.array([r["b"] for r in recs]),
             n=np.array([r["n"] for r in recs]), feats=np.stack([r["feats"] for r in recs]),
             nt=np.array([r["nt"] for r in recs]), ns0=np.array([r["ns0"] for r in recs]),
             np0=np.array([r["np0"] for r in recs]), best_ns=np.array([r["best_ns"] for r in recs]),
             best_np=np.array([r["best_np"] for r in recs]),
             best_time=np.array([r["best_time"] for r in recs]),
             found=np.array([r["found"] for r in recs]), margin=np.array([r["margin"] for r in recs]),
             mvm_best=np.array([r["mvm_best"] for r in recs]),
             runs=np.array(json.dumps([r["runs"] for r in recs])))


L2_FIT = 2e-3        # amplitude penalty of the correction fit (unique, smooth targets)
GAIN_MIN = 0.05      # a sweep point replaces the rule only if it needs this much fewer products


def rule_margin(feats, n, a, b, delta, n_s):
    """delta' of the rule for a given N_S, from the stored moments."""
    mu = np.asarray(feats[:N_MOM], np.float64)
    return B.chebfd_dos_params(mu, int(n), a, b, -delta, delta, n_s=int(n_s), ns_max=NS_MAX,
                               with_margin=True)[3]


def fitted_corrections(a, b, delta, margin, n_p, iters=120):
    amp, sig = B.chebfd_fit_corrections(a, b, -delta, delta, -delta - margin, delta + margin,
                                        int(n_p), n_hat=N_HAT, c_max=C_MAX, iters=iters, l2=L2_FIT)
    return amp, sig


def fit_targets(out_path, inputs):
    """Training targets: log ratios of the sweep's best (N_p, N_S) to the
    rule where the best needs at least GAIN_MIN fewer matrix-vector products
    (else 0: keep the rule), and the hat amplitudes that minimise the damping factor of the
    rule's filter for the rule's search interval (fitted on the host, one
    thread per sample)."""
    from concurrent.futures import ThreadPoolExecutor
    D = [np.load(p, allow_pickle=False) for p in inputs]
    cat = {k: np.concatenate([d[k] for d in D]) for k in D[0].files if k != "runs"}
    runs = sum((json.loads(str(d["runs"])) for d in D), [])
    m = len(cat["seed"])

    def one(i):
        mg = rule_margin(cat["feats"][i], cat["n"][i], cat["a"][i], cat["b"][i], cat["delta"][i],
                         cat["ns0"][i])
        return fitted_corrections(cat["a"][i], cat["b"][i], cat["delta"][i], mg,
                                  cat["np0"][i])[0]

    with ThreadPoolExecutor(max_workers=os.cpu_count() or 4) as ex:
        amps = list(ex.map(one, range(m)))
    T = np.zeros((m, 2 + N_HAT), np.float32)
    for i in range(m):
        m_rule = [r[5] for r in runs[i] if r[0] == cat["ns0"][i] and r[1] == cat["np0"][i]]
        if m_rule and 0 < cat["mvm_best"][i] < (1.0 - GAIN_MIN) * m_rule[0]:
            T[i, 0] = np.log(cat["best_np"][i] / cat["np0"][i])
            T[i, 1] = np.log(cat["best_ns"][i] / cat["ns0"][i])
    T[:, 2:] = np.stack(amps)
    np.savez(out_path, X=cat["feats"].astype(np.float32), T=T, **cat)
    return cat["feats"], T


def train(model_path, data_path, epochs=4000, lr=3e-4, wd=3e-2, val_frac=0.1, seed=1):
    """Full-batch Adam on the GPU with the library's kernels; the parameters
    with the lowest validation loss are kept."""
    import torch
    ctx = B.Context(0)
    D = np.load(data_path, allow_pickle=False)
    X, T = D["X"].astype(np.float32), D["T"].astype(np.float32)
    m = X.shape[0]
    g = np.random.default_rng(seed)
    perm = g.permutation(m)
    nv = max(1, int(round(val_frac * m)))
    vi, ti = perm[:nv], perm[nv:]
    net = B.MLP(ctx, X.shape[1], HIDDEN, T.shape[1], seed=seed)
    shift = T[ti].mean(0)
    scale = np.maximum(T[ti].std(0), 1e-3)
    net.set(shift=shift, scale=scale)
    in_shift = X[ti].mean(0)
    in_scale = np.maximum(X[ti].std(0), 1e-6)
    net.input_scaling(in_shift, in_scale)
    Xt, Tt = torch.from_numpy(X[ti]).cuda(), torch.from_numpy(T[ti]).cuda()
    Xv, Tv = torch.from_numpy(X[vi]).cuda(), torch.from_numpy(T[vi]).cuda()
    best = (math.inf, None, 0)
    hist = []
    for ep in range(epochs):
        lt = net.train_step(Xt, Tt, lr, wd)
        if ep % 10 == 0 or ep == epochs - 1:
            lv, _ = net.loss_grad(Xv, Tv)
            hist.append((ep, lt, lv))
            if lv < best[0]:
                best = (lv, net.get()[0].copy(), ep)
    params = best[1]
    np.savez(model_path, params=params, shift=shift, scale=scale, in_shift=in_shift,
             in_scale=in_scale,
             dims=np.array([X.shape[1], HIDDEN, T.shape[1]]), val_loss=best[0], epoch=best[2],
             history=np.array(hist), val_index=vi)
    print(json.dumps(dict(train_loss=hist[-1][1], best_val_loss=best[0], best_epoch=best[2],
                          n_train=len(ti), n_val=len(vi))), flush=True)
    return model_path


def load_model(ctx, path):
    D = np.load(path, allow_pickle=False)
    n_in, h, n_out = (int(x) for x in D["dims"])
    net = B.MLP(ctx, n_in, h, n_out)
    net.set(params=D["params"], shift=D["shift"], scale=D["scale"])
    net.input_scaling(D["in_shift"], D["in_scale"])
    return net


def gate_corrections(P, n_p, n_s, corr):
    """The plain expansion is the fallback: corrections are kept only if
    they lower the damping factor sigma (Sec. 2.3) of the filter for the
    rule's search interval at this (N_p, N_S); returns corr or None."""
    if corr is None or not np.any(corr):
        return None
    mu = np.asarray(P.get("mu_rule", P["mu"][:N_MOM]), np.float64)
    a, b, d = P["a"], P["b"], P["delta"]
    ns_max = max(NS_MAX, int(n_s))
    margin = B.chebfd_dos_params(mu, int(P["n"]), a, b, -d, d, n_s=int(n_s), ns_max=ns_max,
                                 with_margin=True)[3]
    g = B.chebfd_coeffs(-d, d, a, b, int(n_p))
    s_plain = B.chebfd_filter_quality(g, a, b, -d, d, -d - margin, d + margin)[0]
    s_corr = B.chebfd_filter_quality(g * (1.0 + corr), a, b, -d, d, -d - margin, d + margin)[0]
    return corr if s_corr < s_plain else None


def predict(ctx, net, P, n_s_fixed=0, gate=True):
    """(n_p, n_s, corrections) from the network for problem P; with a fixed
    N_S the rule is re-evaluated for that N_S and only the degree ratio and
    the corrections are taken from the network.  With gate, corrections
    that do not improve the filter's damping factor are dropped."""
    import torch
    Y = net.forward(torch.from_numpy(P["feats"][None, :]).cuda()).cpu().numpy()[0]
    np_ref, ns_ref = P["np0"], P["ns0"]
    if n_s_fixed:
        mu_rule = P.get("mu_rule", P["mu"])
        _, ns_ref, np_ref = B.chebfd_dos_params(mu_rule, P["n"], P["a"], P["b"], -P["delta"],
                                                P["delta"], n_s=n_s_fixed, ns_max=max(NS_MAX, n_s_fixed))
        Y = Y.copy()
        Y[1] = 0.0
    n_p, n_s, corr = B.chebfd_learned_decode(Y, np_ref, ns_ref, N_HAT, C_MAX,
                                             ns_max=max(NS_MAX, n_s_fixed))
    if gate:
        corr = gate_corrections(P, n_p, n_s, corr)
    return n_p, n_s, corr


def evaluate(out_path, model_path, seeds):
    """Held-out comparison: rule-based parameters vs the network's, both
    solved to residual 1e-9 with the plain FP64 solver."""
    ctx = B.Context(0)
    net = load_model(ctx, model_path)
    rows = []
    for s in seeds:
        P = problem(ctx, s)
        base = run_solve(ctx, P["H"], P["delta"], P["ns0"], P["np0"], seed=s)
        n_p, n_s, corr = predict(ctx, net, P)
        lrn = run_solve(ctx, P["H"], P["delta"], n_s, n_p, corr=corr, seed=s)
        # reference point: the rule with corrections fitted for this sample
        mg = rule_margin(P["feats"], P["n"], P["a"], P["b"], P["delta"], P["ns0"])
        amp, _ = fitted_corrections(P["a"], P["b"], P["delta"], mg, P["np0"])
        _, _, cfit = B.chebfd_learned_decode(np.r_[0.0, 0.0, amp].astype(np.float32), P["np0"],
                                             P["ns0"], N_HAT, C_MAX, ns_max=NS_MAX)
        fit = run_solve(ctx, P["H"], P["delta"], P["ns0"], P["np0"], corr=cfit, seed=s)
        same = base["found"] == lrn["found"] and (base["found"] == 0 or np.abs(
            base["evals"] - lrn["evals"]).max() < 1e-10 * max(abs(P["a"]), abs(P["b"])))
        row = dict(seed=s, W=P["W"], delta=P["delta"], found_rule=base["found"],
                   found_learned=lrn["found"], same_eigenvalues=bool(same),
                   time_rule=base["time"], time_learned=lrn["time"], mvm_rule=base["n_mvm"],
                   mvm_learned=lrn["n_mvm"], rule=(P["ns0"], P["np0"]), learned=(n_s, n_p),
                   time_fitted_corr=fit["time"], mvm_fitted_corr=fit["n_mvm"],
                   found_fitted_corr=fit["found"], iters_rule=base["iterations"],
                   iters_learned=lrn["iterations"], iters_fitted_corr=fit["iterations"],
                   max_res_rule=float(base["res"].max()) if base["found"] else None,
                   max_res_learned=float(lrn["res"].max()) if lrn["found"] else None)
        rows.append(row)
        print(json.dumps(row), flush=True)
    t_r = sum(r["time_rule"] for r in rows)
    t_l = sum(r["time_learned"] for r in rows)
    t_f = sum(r["time_fitted_corr"] for r in rows)
    summary = dict(n=len(rows), total_time_rule=t_r, total_time_learned=t_l,
                   speedup=t_r / t_l, all_same=all(r["same_eigenvalues"] for r in rows),
                   mvm_ratio=sum(r["mvm_rule"] for r in rows) / max(1, sum(r["mvm_learned"] for r in rows)),
                   total_time_fitted_corr=t_f, speedup_fitted_corr=t_r / t_f,
                   mvm_ratio_fitted_corr=sum(r["mvm_rule"] for r in rows) / max(1, sum(r["mvm_fitted_corr"] for r in rows)))
    with open(out_path, "w") as fh:
        json.dump(dict(summary=summary, rows=rows), fh, indent=1)
    print(json.dumps(summary), flush=True)
    return summary


def main(argv):
    cmd = argv[0]
    if cmd == "sweep":
        sweep(argv[1], range(int(argv[2]), int(argv[3])))
    elif cmd == "fit":
        fit_targets(argv[1], argv[2:])
    elif cmd == "train":
        train(argv[1], argv[2])
    elif cmd == "eval":
        evaluate(argv[1], argv[2], range(int(argv[3]), int(argv[4])))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
