"""Benchmark: fused Chebyshev SpMMV throughput on one MI355X, and time to
all window eigenpairs (residual < 1e-9).

    python bench.py [--steps K] [--warmup W] [--workload ti_256x256x64]
                    [--storage sell|stencil] [--precision c128|c64]
                    [--kernel-only] [--no-cpu-baseline]

Headline (the largest single-GPU lattice, 256x256x64, N = 16,777,216, 128
search vectors in complex128, the lattice Hamiltonian applied matrix-free;
`kernels` gives the same step on the stored SELL-32-256 matrix and both in
complex64): a step is one fused launch of the Chebyshev filter (Fig.
fig:ChebFD: the sparse matrix-multiple-vector product fused with the
three-term recurrence and the filter accumulation, Sec. 4), with the matrix
(or the site potentials) and the three blocks resident in HBM.  The timed
region is one filter application of degree K, i.e. exactly K fused launches
(the first two set up the recurrence); `value` is their algorithmic bytes
(the matrix once, u read once, w and x read and written, per launch)
divided by the region's wall time.  The `roofline` object gives the plain
recurrence launch alone: its HIP-event duration is the difference of the
degree-K and degree-2 applications over K - 2, on the library's stream.
A complete solve at this size takes 700-1000 s, so time to all window
eigenpairs is reported from the 128x128x64 lattice (precision form and FP64
form on Lanczos bounds) and the 64x64x32 lattice (FP64).  Prints one JSON
line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import chebfd_inputs as inp  # noqa: E402

HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = {"sell": ["kernels_step.hip", "pack.h", "dispatch.h", "matrix.cpp"],
                  "stencil": ["kernels_stencil.hip", "pack.h", "dispatch.h", "matrix.cpp"]}
METRIC = "fused Chebyshev SpMMV GB/s vs HBM peak; time to all window eigenpairs @res<1e-9"


def source_sha(storage):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[storage]:
        with open(os.path.join(ROOT, "paper_1510_04895_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def step_flops(n, n_b, nnz_row):
    """Flops of one fused step with the paper's complex counting (Sec. 4.2):
    N_nzr (F_a + F_m) + ceil(9 F_a/2) + ceil(11 F_m/2) per row and vector,
    F_a = 2, F_m = 6."""
    return n * n_b * (nnz_row * 8 + 42)


def measured_traffic(storage, precision, workload):
    """HBM bytes per fused launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{storage}_{precision}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_source_sha") != source_sha(storage):
        return None
    return t


def host_info():
    model, mem = platform.processor() or "unknown", None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as fh:
            for line in fh:
                if line.startswith("MemTotal"):
                    mem = round(int(line.split()[1]) / 2**20, 1)
                    break
    except OSError:
        pass
    return model, mem


def cpu_baseline(L, n_s, target_s=15.0, max_steps=400):
    """The oracle's filter (plain CSR, OpenMP static over the host threads)
    on an 8-layer slab of the lattice (same x-y extent and block width as
    the GPU figure; the full lattice's blocks do not fit host memory), timed
    on the host cores.  The number of recurrence steps is chosen from a
    two-step probe so that the timed sample takes about target_s seconds."""
    import oracle
    Ls = (L[0], L[1], min(L[2], 8))
    H = oracle.ti_hamiltonian(*Ls, pbc=3, V=1.0, seed=1)
    a, b = oracle.gershgorin(H)
    X = inp.random_block(H.n, n_s, seed=1)
    d = 0.02 * max(abs(a), abs(b))
    t0 = time.perf_counter()
    oracle.filter_block(H, a, b, oracle.gamma(-d, d, a, b, 2), X)
    per_step = (time.perf_counter() - t0) / 2
    n_steps = int(min(max_steps, max(3, target_s / max(per_step, 1e-6))))
    gam = oracle.gamma(-d, d, a, b, n_steps)
    t0 = time.perf_counter()
    oracle.filter_block(H, a, b, gam, X)
    dt = time.perf_counter() - t0
    vb = H.nnz * 20 + 5 * H.n * n_s * 16
    model, mem = host_info()
    # the oracle's complete solve (Sec. 3.1 steps 1-8) of the 8x8x8
    # correctness configuration, beside the library's time_to_solution entry
    w8, d8 = solve_8x8x8_window()
    H8 = oracle.ti_hamiltonian(8, 8, 8, pbc=3, V=1.0, seed=1)
    t0 = time.perf_counter()
    rc8, ev8, _, _, _ = oracle.chebfd_solve(H8, -d8, d8, 32, 200, seed=1001, vectors=False)
    t8 = time.perf_counter() - t0
    solve8 = dict(time_to_solution_s=round(t8, 3), status=int(rc8), eigenpairs_found=int(ev8.size),
                  config="8x8x8, window of the 16 dense eigenvalues nearest 0, n_s 32, n_p 200, "
                         "Gershgorin bounds, FP64")
    return dict(value=round(n_steps * vb / dt / 1e9, 3), unit="GB/s", cores=oracle.num_threads(),
                kind="oracle", cpu_model=model, host_mem_gib=mem, solve_8x8x8=solve8,
                sample=f"filter of degree {n_steps} ({n_steps} recurrence steps of Fig. "
                       f"fig:ChebFD, CSR, OpenMP static) on the {Ls[0]}x{Ls[1]}x{Ls[2]} slab of "
                       f"the lattice (N={H.n}), n_s={n_s}, c128, {dt:.1f} s on "
                       f"{oracle.num_threads()} threads; bytes per step nnz*20 + 5*N*n_s*16, "
                       f"as for the GPU figure")


def solve_8x8x8_window():
    """The golden dense spectrum of the 8x8x8 lattice (seed 1) and the
    half-width that holds its 16 eigenvalues nearest 0."""
    w = np.loadtxt(os.path.join(ROOT, "tests", "golden", "ti_8x8x8_V1_seed1_evals.txt"))
    aw = np.sort(np.abs(w))
    return w, 0.5 * (aw[15] + aw[16])


def launch_bytes(mat, n, n_s, s_d, k):
    """Algorithmic bytes of a degree-k filter application: the first launch
    reads u and writes w, the second reads u and x and writes w and x, each
    later one reads u, w, x and writes w, x; every launch reads the matrix."""
    blk = n * n_s * s_d
    return k * mat + blk * (2 + 4 + 5 * (k - 2))


class Blocks:
    """The three device blocks of the filter, allocated once per precision."""

    def __init__(self, torch, B, ctx, n, n_s, prec):
        dt = torch.complex128 if prec == B.PREC_C128 else torch.complex64
        self.X = torch.empty((n, n_s), dtype=dt, device="cuda")
        self.U = torch.empty_like(self.X)
        self.W = torch.empty_like(self.X)
        B.chebfd_random_block(ctx, self.X, seed=7)


def time_filter(torch, B, ctx, H, blocks, gam, a, b):
    """HIP-event and wall time of one filter application on the library's
    stream (the context runs on torch's current stream)."""
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record(stream)
    B.chebfd_filter_apply(ctx, H, gam, a, b, blocks.X, blocks.U, blocks.W)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3, time.perf_counter() - w0


def step_time(torch, B, ctx, H, blocks, a, b, k):
    """Average duration of one plain recurrence launch: (t(degree k) -
    t(degree 2)) / (k - 2), the degree-2 time the median of three."""
    d = 0.02 * max(abs(a), abs(b))
    gk = B.chebfd_coeffs(-d, d, a, b, k)
    time_filter(torch, B, ctx, H, blocks, gk[:3].copy(), a, b)   # warm-up
    tk = time_filter(torch, B, ctx, H, blocks, gk, a, b)[0]
    t2 = sorted(time_filter(torch, B, ctx, H, blocks, gk[:3].copy(), a, b)[0] for _ in range(3))
    return (tk - t2[1]) / (k - 2)


def solve_case(torch, B, ctx, wname, storage, prec, bounds, tag, polish=None):
    """One complete solve (Sec. 3.1 steps 1-8) on a lattice with its window
    from the workload table; returns a summary dict and the eigenvalues."""
    w = inp.WORKLOADS[wname]
    st = B.STORAGE_SELL if storage == "sell" else B.STORAGE_STENCIL
    torch.cuda.synchronize()
    tb = time.perf_counter()
    H = B.Matrix.ti(ctx, w["L"], pbc=w["pbc"], V=w["V"], seed=w["seeds"][0], storage=st,
                    sell_C=w.get("sell_C", 32), sell_sigma=w.get("sell_sigma", 256))
    torch.cuda.synchronize()
    t_build = time.perf_counter() - tb
    info = H.info()
    steps = 40 if bounds == "lanczos" else 0
    a, b = (B.chebfd_lanczos_bounds(ctx, H, k=40, seed=w["seeds"][0]) if steps
            else (info["g_lo"], info["g_hi"]))
    d = w["delta"]
    dp = d * (math.sqrt(w["n_s"] / w["n_target"]) - 1.0)
    n_p, eta = B.chebfd_optimal_np(a, b, -d, d, -d - dp, d + dp)
    p = B.default_params(lam_lo=-d, lam_hi=d, n_s=w["n_s"], n_p=n_p, kernel=w["kernel"],
                         mu=w["mu"], eps=w["eps"], max_iter=60, precision=prec, lock=1,
                         seed=w["seeds"][0], vectors=0, bounds=steps,
                         polish=B.POLISH_CORRECTION if polish is None else polish)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, ev, rs, _, stats = B.chebfd_solve(ctx, H, p)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    del H
    torch.cuda.empty_cache()
    out = {"workload": wname, "storage": storage,
           "precision": ("c128" if prec == B.PREC_C128
                         else "c64 sweep + FP64 filter polish" if polish == B.POLISH_FP64
                         else "c64 sweep + FP32 correction polish (FP64 accuracy)"),
           "bounds": [round(a, 4), round(b, 4), bounds], "window": [-d, d], "n_s": w["n_s"],
           "n_p": n_p, "time_to_solution_s": round(T, 3), "matrix_build_s": round(t_build, 3),
           "status": int(rc),
           "eigenpairs_found": int(ev.size), "max_residual": float(rs.max()) if rs.size else None,
           "iterations": stats["iterations"], "iterations_c64": stats["iterations_c64"],
           "iterations_correction": stats["iterations_corr"],
           "n_mvm": stats["n_mvm"], "t_filter_s": round(stats["t_filter"], 3),
           "t_ortho_s": round(stats["t_ortho"], 3), "t_rr_s": round(stats["t_rr"], 3)}
    if prec != B.PREC_C128 and stats["sweep_evals"].size:
        out["sweep_pairs"] = int(stats["sweep_evals"].size)
        out["sweep_max_residual"] = float(stats["sweep_residuals"].max())
    print(f"# solve {tag}: {T:.2f} s, {ev.size} pairs, max residual "
          f"{out['max_residual']}", flush=True)
    return out, ev


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40,
                    help="fused launches in the timed region (one filter of this degree)")
    ap.add_argument("--warmup", type=int, default=5, help="untimed fused launches first")
    ap.add_argument("--workload", default="ti_256x256x64")
    ap.add_argument("--storage", default="stencil", choices=["sell", "stencil"])
    ap.add_argument("--precision", default="c128", choices=["c128", "c64"])
    ap.add_argument("--order", type=int, default=-1, choices=[-1, 0, 1],
                    help="block order of the matrix-free step (tuning key 'order'): -1 "
                         "automatic, 0 column-slab major, 1 tiled lattice order")
    ap.add_argument("--lanes", type=int, default=0, choices=[0, 16, 32, 64],
                    help="lanes per row or site (tuning key 'lanes'; 0 = automatic)")
    ap.add_argument("--tile", type=int, default=-1,
                    help="strip width of the tiled lattice order (tuning key 'tile'; -1 = default)")
    ap.add_argument("--kernel-only", action="store_true",
                    help="only the bandwidth probe and the timed fused launches (no solves)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-other", action="store_true",
                    help="skip the other storage and the other precision's kernel timings")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); sharding across GPUs "
              "is designed but not built", file=sys.stderr)
        sys.exit(2)
    if args.steps < 3:
        sys.exit("bench.py: --steps must be >= 3")

    import torch
    from paper_1510_04895_amd import binding as B

    w = inp.WORKLOADS[args.workload]
    L = w["L"]
    n_s = w["n_s"]
    ctx = B.Context(0)
    if args.order != -1:
        B.chebfd_set_tuning(ctx, "order", args.order)
    if args.lanes:
        B.chebfd_set_tuning(ctx, "lanes", args.lanes)
    if args.tile != -1:
        B.chebfd_set_tuning(ctx, "tile", args.tile)
    prec = B.PREC_C128 if args.precision == "c128" else B.PREC_C64

    # attainable bandwidth (read-only reduction, copy, 3-read/2-write stream)
    buf = torch.empty(4 * 2**30, dtype=torch.uint8, device="cuda")
    probe = B.chebfd_bandwidth_probe(ctx, buf, reps=5)
    del buf
    torch.cuda.empty_cache()
    print(f"# probe GB/s read {probe[0]:.0f} copy {probe[1]:.0f} 3r2w {probe[2]:.0f}", flush=True)

    mats, kern = {}, {}
    for storage in [args.storage] + ([] if args.no_other else
                                     [s for s in ("sell", "stencil") if s != args.storage]):
        st = B.STORAGE_SELL if storage == "sell" else B.STORAGE_STENCIL
        t0 = time.perf_counter()
        mats[storage] = B.Matrix.ti(ctx, L, pbc=w["pbc"], V=w["V"], seed=w["seeds"][0],
                                    storage=st, sell_C=w.get("sell_C", 32),
                                    sell_sigma=w.get("sell_sigma", 256))
        print(f"# matrix {storage} built in {time.perf_counter() - t0:.2f} s", flush=True)
    info = mats[args.storage].info()
    n, nnz = info["n"], info["nnz"]
    a, b = info["g_lo"], info["g_hi"]

    def mat_bytes(storage, p):
        i = mats[storage].info()
        return i["matrix_bytes_c128"] if p == B.PREC_C128 else i["matrix_bytes_c64"]

    precs = [prec] + ([] if args.no_other else
                      [B.PREC_C64 if prec == B.PREC_C128 else B.PREC_C128])
    headline = None
    for pr in precs:
        s_d = 16 if pr == B.PREC_C128 else 8
        blocks = Blocks(torch, B, ctx, n, n_s, pr)
        for storage in mats:
            H = mats[storage]
            vstep = mat_bytes(storage, pr) + 5 * n * n_s * s_d
            if storage == args.storage and pr == prec:
                d = 0.02 * max(abs(a), abs(b))
                # warm-up, then exactly K fused launches (one filter of degree K)
                time_filter(torch, B, ctx, H, blocks,
                            B.chebfd_coeffs(-d, d, a, b, max(args.warmup, 2)), a, b)
                gk = B.chebfd_coeffs(-d, d, a, b, args.steps)
                t_ev, t_wall = time_filter(torch, B, ctx, H, blocks, gk, a, b)
                t2 = sorted(time_filter(torch, B, ctx, H, blocks, gk[:3].copy(), a, b)[0]
                            for _ in range(3))
                t_step = (t_ev - t2[1]) / (args.steps - 2)
                headline = dict(t_wall=t_wall, t_ev=t_ev, t_step=t_step, vstep=vstep,
                                vk=launch_bytes(mat_bytes(storage, pr), n, n_s, s_d, args.steps))
            else:
                t_step = step_time(torch, B, ctx, H, blocks, a, b, 22)
            key = f"{storage}_{'c128' if pr == B.PREC_C128 else 'c64'}"
            kern[key] = {"avg_launch_us": round(t_step * 1e6, 2),
                         "algorithmic_bytes_per_launch": int(vstep),
                         "achieved_gbs": round(vstep / t_step / 1e9, 1),
                         "frac": round(vstep / t_step / 1e9 / HBM_PEAK_GBS, 4)}
            print(f"# {key}: fused launch {t_step * 1e6:.1f} us = {vstep / t_step / 1e9:.0f} "
                  f"GB/s", flush=True)
        del blocks
        torch.cuda.empty_cache()
    mats.clear()
    torch.cuda.empty_cache()

    # the committed counters were taken in the default launch shape
    default_shape = args.order == -1 and not args.lanes and args.tile == -1
    traffic = measured_traffic(args.storage, args.precision, args.workload) if default_shape else None
    t_step = headline["t_step"]
    roof = {"bound": "hbm", "achieved": round(headline["vstep"] / t_step / 1e9, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(headline["vstep"] / t_step / 1e9 / HBM_PEAK_GBS, 4),
            "traffic": (int(traffic["fetch_bytes"] + traffic["write_bytes"]) if traffic else None),
            "kernel": ("k_step_sell" if args.storage == "sell" else "k_step_ti") + " (MODE_STEP)",
            "algorithmic_bytes_per_launch": int(headline["vstep"]),
            "avg_launch_us": round(t_step * 1e6, 2),
            "frac_of_probe_3r2w": round(headline["vstep"] / t_step / 1e9 / probe[2], 4)}
    cfg = {"workload": args.workload, "lattice": "x".join(map(str, L)), "N": n, "nnz": nnz,
           "n_s": n_s, "storage": args.storage, "order": args.order, "lanes": args.lanes,
           "tile": args.tile,
           "sell_C_sigma": [w.get("sell_C", 32), w.get("sell_sigma", 256)]
           if args.storage == "sell" else None,
           "step": "one fused Chebyshev launch (spMMV + recurrence + accumulation)",
           "bounds": [round(a, 4), round(b, 4), "gershgorin"]}
    out = {"metric": METRIC, "value": round(headline["vk"] / headline["t_wall"] / 1e9, 2),
           "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(headline["t_wall"] / args.steps * 1e3, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if prec == B.PREC_C128 else "f32", "data": "synthetic",
           "config": cfg,
           "timed_region_event_s": round(headline["t_ev"], 5),
           "fused_kernel_tflops": round(step_flops(n, n_s, nnz / n) / t_step / 1e12, 3),
           "kernels": kern,
           # the paper's own filter-step rate on a CPU cluster (Table
           # tab:benchmark, largest TI run): another machine and a 64x larger
           # matrix, so context for the flop/s figure, not a target
           "paper_context": {"value": 43.9, "unit": "Tflop/s", "per_node": 0.0857,
                             "system": "512 CPU nodes, two 14-core Xeon E5-2697v3 each",
                             "workload": "TI matrix, D = 1.07e9, N_S = 256, N_p = 8639",
                             "flop_convention": "same complex counting (Sec. 4.2)"}}

    if not args.kernel_only:
        # time to all window eigenpairs: the precision form (with FP32
        # correction passes, and with FP64 passes in the polish) against the
        # FP64 form at 128x128x64 (Lanczos bounds), the FP64 solve at
        # 64x64x32 and at 8x8x8
        tts = {}
        r64, ev64 = solve_case(torch, B, ctx, "ti_128x128x64", args.storage, B.PREC_C128,
                               "lanczos", "128x128x64 c128")
        r32, ev32 = solve_case(torch, B, ctx, "ti_128x128x64", args.storage, B.PREC_C64,
                               "lanczos", "128x128x64 c64")
        S_w = max(abs(r64["bounds"][0]), abs(r64["bounds"][1]))
        r32["same_eigenvalues_as_fp64"] = bool(
            ev32.size == ev64.size and (ev64.size == 0 or
                                        np.abs(ev32 - ev64).max() < 1e-10 * S_w))
        r32["speedup_over_fp64"] = round(r64["time_to_solution_s"] / r32["time_to_solution_s"], 3)
        tts["ti_128x128x64_fp64"] = r64
        tts["ti_128x128x64_precision_form"] = r32
        # the same precision form with FP64 filter passes in the polish
        rp, evp = solve_case(torch, B, ctx, "ti_128x128x64", args.storage, B.PREC_C64,
                             "lanczos", "128x128x64 c64, FP64 polish", polish=B.POLISH_FP64)
        rp["same_eigenvalues_as_fp64"] = bool(
            evp.size == ev64.size and (ev64.size == 0 or
                                       np.abs(evp - ev64).max() < 1e-10 * S_w))
        rp["speedup_over_fp64"] = round(r64["time_to_solution_s"] / rp["time_to_solution_s"], 3)
        tts["ti_128x128x64_precision_form_fp64_polish"] = rp
        r2, ev2 = solve_case(torch, B, ctx, "ti_64x64x32", args.storage, B.PREC_C128,
                             "gershgorin", "64x64x32 c128")
        gold = os.path.join(ROOT, "tests", "golden", "ti_64x64x32_V1_seed1_window0.23.txt")
        if os.path.exists(gold):
            g = np.sort(np.loadtxt(gold)[:, 0])
            g = g[np.abs(g) <= r2["window"][1]]
            S2 = max(abs(r2["bounds"][0]), abs(r2["bounds"][1]))
            r2["matches_oracle_window"] = bool(g.size == ev2.size and
                                               np.abs(g - ev2).max() < 1e-10 * S2)
        tts["ti_64x64x32_fp64"] = r2
        # the 8x8x8 correctness configuration (the CPU leg times the
        # oracle's solve of the same configuration)
        w8, d8 = solve_8x8x8_window()
        H8 = B.Matrix.ti(ctx, (8, 8, 8), pbc=3, V=1.0, seed=1, storage=(B.STORAGE_SELL if args.storage == "sell"
                                          else B.STORAGE_STENCIL))
        p8 = B.default_params(lam_lo=-d8, lam_hi=d8, n_s=32, n_p=200, eps=1e-9, seed=1001,
                              vectors=0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc8, ev8, rs8, _, st8 = B.chebfd_solve(ctx, H8, p8)
        torch.cuda.synchronize()
        t8 = time.perf_counter() - t0
        want = np.sort(w8[np.abs(w8) <= d8])
        S8 = max(abs(st8["a"]), abs(st8["b"]))
        tts["ti_8x8x8_fp64"] = {
            "time_to_solution_s": round(t8, 4), "status": int(rc8),
            "eigenpairs_found": int(ev8.size), "iterations": st8["iterations"],
            "max_residual": float(rs8.max()) if rs8.size else None,
            "matches_dense_oracle": bool(ev8.size == want.size and
                                         np.abs(ev8 - want).max() < 1e-10 * S8)}
        del H8
        out["time_to_solution"] = tts
    out["roofline"] = roof
    out["bandwidth_probe_gbs"] = {"read_only": round(probe[0], 1), "copy": round(probe[1], 1),
                                  "stream_3r2w": round(probe[2], 1)}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(L, n_s)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
