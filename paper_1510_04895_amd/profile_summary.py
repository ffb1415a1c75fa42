"""Turns rocprofv3 CSV output into the short summaries kept under profiles/.

    python -m paper_1510_04895_amd.profile_summary stats KERNEL_STATS_CSV NAME "COMMAND"
        -> profiles/NAME.md: per-kernel calls / average / total / share.
    python -m paper_1510_04895_amd.profile_summary traffic STORAGE PREC WORKLOAD \\
           FETCH_DIR WRITE_DIR "FETCH_COMMAND" "WRITE_COMMAND" [NAME]
        -> profiles/traffic_STORAGE_PREC_WORKLOAD.json (or NAME.json for another
           launch shape): HBM bytes per fused
           MODE_STEP launch from FETCH_SIZE / WRITE_SIZE (KiB per dispatch),
           each scaled by what the same counter reads for the plain copy
           kernel of the bandwidth probe (2 GiB read + 2 GiB written), with
           the hash of the kernel sources the counters were taken on.
    python -m paper_1510_04895_amd.profile_summary mfma PMC_DIR NAME "COMMAND"
        -> profiles/NAME.md: per MFMA kernel, the FP64 MFMA flops per dispatch
           (SQ_INSTS_VALU_MFMA_MOPS_F64 x 512) and the MFMA busy share of all
           SIMD cycles (SQ_VALU_MFMA_BUSY_CYCLES over the GPU-active cycles
           times the SIMD count; the CSV carries GRBM_GUI_ACTIVE summed over
           the XCDs, each of which counts the same cycles).
"""
from __future__ import annotations

import collections
import csv
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 2 * 2**30    # bytes the probe's copy kernel reads (and writes)


def _pmc(path):
    agg = collections.defaultdict(list)
    with open(path) as fh:
        for r in csv.DictReader(fh):
            agg[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return agg


def _mode(name):
    """MODE template argument of a fused-step kernel name (k_step_sellg
    carries the row-group size before it)."""
    m = re.search(r"k_step_sellg<[^,]+, \d+, \d+, \d+, (\d)", name)
    if m:
        return int(m.group(1))
    m = re.search(r"k_step_(sell|ti)<[^,]+, \d+, \d+, (\d)", name)
    return int(m.group(2)) if m else None


def _csv_in(d):
    for dp, _, fs in os.walk(d):
        for f in fs:
            if f.endswith("counter_collection.csv"):
                return os.path.join(dp, f)
    raise FileNotFoundError(d)


def traffic(storage, prec, workload, fdir, wdir, cmd_f, cmd_w, name=None):
    sys.path.insert(0, ROOT)
    import bench
    F, Wc = _pmc(_csv_in(fdir)), _pmc(_csv_in(wdir))
    cf = [v for k, vs in F.items() if "k_copy16" in k for v in vs]
    cw = [v for k, vs in Wc.items() if "k_copy16" in k for v in vs]
    f_scale = COPY_BYTES / (sum(cf) / len(cf) * 1024)
    w_scale = COPY_BYTES / (sum(cw) / len(cw) * 1024)
    fs = [v for k, vs in F.items() if _mode(k) == 2 for v in vs]
    ws = [v for k, vs in Wc.items() if _mode(k) == 2 for v in vs]
    out = dict(storage=storage, precision=prec, workload=workload,
               kernel_mode="MODE_STEP (w = 2(aH+b)u - w; x += g w)", dispatches=len(fs),
               fetch_bytes=sum(fs) / len(fs) * 1024 * f_scale,
               write_bytes=sum(ws) / len(ws) * 1024 * w_scale, fetch_scale=f_scale,
               write_scale=w_scale, kernel_source_sha=bench.source_sha(storage),
               commands=[cmd_f, cmd_w])
    # the default name is the record bench.py reads (default launch shape);
    # counters of another launch shape take a name of their own
    name = name or f"traffic_{storage}_{prec}_{workload}"
    path = os.path.join(ROOT, "profiles", f"{name}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    return out


SIMDS = 256 * 4             # MI355X: 256 compute units of 4 SIMDs
XCDS = 8                    # GRBM_GUI_ACTIVE arrives summed over the 8 XCDs


def mfma(pmc_dir, name, cmd, kernels=("k_gram", "k_block_times")):
    vals = collections.defaultdict(list)
    per_disp = collections.defaultdict(float)   # (kernel, dispatch) -> MFMA ops
    with open(_csv_in(pmc_dir)) as fh:
        for r in csv.DictReader(fh):
            vals[(r["Kernel_Name"], r["Counter_Name"])].append(float(r["Counter_Value"]))
            if r["Counter_Name"] == "SQ_INSTS_VALU_MFMA_MOPS_F64":
                per_disp[(r["Kernel_Name"], r["Dispatch_Id"])] += float(r["Counter_Value"])
    lines = [f"# {name}", "", "Command (from the repository root, TMPDIR=/tmp):", "",
             "    " + cmd, "",
             "| kernel | dispatches | FP64 MFMA flops per dispatch (mean) | largest dispatch | "
             "MFMA busy, % of SIMD cycles |",
             "|---|---:|---:|---:|---:|"]
    out = {}
    for (k, c), v in sorted(vals.items()):
        if c != "SQ_INSTS_VALU_MFMA_MOPS_F64" or not any(s in k for s in kernels):
            continue
        busy = sum(vals[(k, "SQ_VALU_MFMA_BUSY_CYCLES")])
        gui = sum(vals[(k, "GRBM_GUI_ACTIVE")])
        disp = [f for (kk, _), f in per_disp.items() if kk == k]
        flops = sum(disp) * 512 / len(disp)
        fmax = max(disp) * 512
        util = 100.0 * busy / (gui / XCDS * SIMDS) if gui > 0 else float("nan")
        nm = k.replace("chebfd::(anonymous namespace)::", "").replace("void ", "").split("(")[0]
        out[nm] = dict(dispatches=len(disp), flops_per_dispatch=flops, flops_max=fmax,
                       mfma_busy_pct=util)
        lines.append(f"| `{nm}` | {len(disp)} | {flops:.4e} | {fmax:.4e} | {util:.1f} |")
    text = "\n".join(lines) + "\n"
    with open(os.path.join(ROOT, "profiles", f"{name}.md"), "w") as fh:
        fh.write(text)
    return out


def stats(path, name, cmd):
    with open(path) as fh:
        rows = list(csv.DictReader(fh))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = [f"# {name}", "", "Command (from the repository root, TMPDIR=/tmp):", "",
             "    " + cmd, "", "| kernel | calls | avg us | total ms | % |",
             "|---|---:|---:|---:|---:|"]
    for r in rows[:16]:
        nm = r["Name"].replace("chebfd::(anonymous namespace)::", "").replace("void ", "")
        nm = nm.split("(")[0]
        lines.append(f"| `{nm}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.1f} | {float(r['Percentage']):.2f} |")
    lines.append(f"\nTotal kernel time: {tot / 1e6:.1f} ms.")
    text = "\n".join(lines) + "\n"
    with open(os.path.join(ROOT, "profiles", f"{name}.md"), "w") as fh:
        fh.write(text)
    return text


if __name__ == "__main__":
    what = sys.argv[1]
    if what == "stats":
        print(stats(*sys.argv[2:5]))
    elif what == "traffic":
        print(json.dumps(traffic(*sys.argv[2:10]), indent=1))
    elif what == "mfma":
        print(json.dumps(mfma(*sys.argv[2:5]), indent=1))
    else:
        raise SystemExit(__doc__)
