"""CPU checks of the measurement tooling: the counter summary's calibration
against the plain copy kernel, the kernel-source hash guard on stored
traffic figures, and the paper's flop count of a fused step (Sec. 4.2)."""
import csv
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _write_pmc(d, rows):
    """rocprofv3 counter CSV rows (kernel, counter, value), one dispatch each."""
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                           "Counter_Value"])
        w.writeheader()
        for i, (k, c, v) in enumerate(rows):
            w.writerow(dict(Dispatch_Id=i + 1, Kernel_Name=k, Counter_Name=c, Counter_Value=v))


def test_traffic_calibration(tmp_path, monkeypatch):
    from paper_1510_04895_amd import profile_summary as ps
    step = "void chebfd::(anonymous namespace)::k_step_sell<double, 32, 1, 2, false, true, true, 16, 5>(...)"
    # the copy kernel reads 2 GiB: FETCH_SIZE reports half, WRITE_SIZE all (KiB)
    _write_pmc(tmp_path / "f", [("k_copy16(...)", "FETCH_SIZE", 2**30 / 1024 / 2),
                                (step, "FETCH_SIZE", 4e6), (step, "FETCH_SIZE", 6e6)])
    _write_pmc(tmp_path / "w", [("k_copy16(...)", "WRITE_SIZE", 2 * 2**30 / 1024),
                                (step, "WRITE_SIZE", 1e6)])
    monkeypatch.setattr(ps, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "profiles")
    monkeypatch.syspath_prepend(ROOT)
    out = ps.traffic("sell", "c128", "w", str(tmp_path / "f"), str(tmp_path / "w"), "cf", "cw")
    assert out["fetch_scale"] == pytest.approx(4.0)
    assert out["write_scale"] == pytest.approx(1.0)
    assert out["fetch_bytes"] == pytest.approx(5e6 * 1024 * 4.0)
    assert out["write_bytes"] == pytest.approx(1e6 * 1024)
    assert out["dispatches"] == 2
    assert json.load(open(tmp_path / "profiles" / "traffic_sell_c128_w.json"))["commands"] == ["cf", "cw"]


def test_stored_traffic_needs_current_kernel_source(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "profiles")
    # copy the kernel sources so the hash can be computed under tmp_path
    src = os.path.join(ROOT, "paper_1510_04895_amd", "csrc")
    os.makedirs(tmp_path / "paper_1510_04895_amd" / "csrc")
    for f in set(sum(bench.KERNEL_SOURCES.values(), [])):
        with open(os.path.join(src, f), "rb") as a, \
                open(tmp_path / "paper_1510_04895_amd" / "csrc" / f, "wb") as b:
            b.write(a.read())
    t = dict(fetch_bytes=1.0, write_bytes=2.0, kernel_source_sha=bench.source_sha("sell"))
    with open(tmp_path / "profiles" / "traffic_sell_c128_x.json", "w") as fh:
        json.dump(t, fh)
    assert bench.measured_traffic("sell", "c128", "x")["write_bytes"] == 2.0
    t["kernel_source_sha"] = "0" * 16
    with open(tmp_path / "profiles" / "traffic_sell_c128_x.json", "w") as fh:
        json.dump(t, fh)
    assert bench.measured_traffic("sell", "c128", "x") is None
    assert bench.measured_traffic("stencil", "c128", "x") is None


def test_step_flops_paper_convention():
    """N N_S (N_nzr (F_a + F_m) + ceil(9 F_a / 2) + ceil(11 F_m / 2)) with
    complex F_a = 2, F_m = 6 (Sec. 4.2)."""
    sys.path.insert(0, ROOT)
    import bench
    F_a, F_m = 2, 6
    per = 13 * (F_a + F_m) + -(-9 * F_a // 2) + -(-11 * F_m // 2)
    assert bench.step_flops(10, 3, 13) == 10 * 3 * per


def test_kpm_window_count_on_the_chebyshev_density():
    """mu_m = delta_{m0} is the density 1/(pi sqrt(1 - x^2)) on [-1, 1]; the
    count of Eq. DOS:target in [-d, d] is N (2/pi) asin(d), and the window
    search inverts it."""
    import math
    import numpy as np
    from paper_1510_04895_amd import scale_runs as sr
    mu = np.zeros(4096)
    mu[0] = 1.0
    n = 1_000_000
    for d in (0.05, 0.2, 0.6):
        want = n * 2.0 / math.pi * math.asin(d)
        assert sr.kpm_count(mu, n, -1.0, 1.0, d) == pytest.approx(want, rel=2e-3)
    d = sr.window_for_count(mu, n, -1.0, 1.0, 100000)
    assert n * 2.0 / math.pi * math.asin(d) == pytest.approx(100000, rel=2e-3)


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU; asked for more it exits with status 2
    and says so, before touching a device."""
    import subprocess
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""



def test_mfma_summary(tmp_path, monkeypatch):
    """FP64 MFMA flops = MOPS x 512 per dispatch; busy share = busy cycles
    summed over SIMDs over (GPU-active cycles x 1024 SIMDs), the active
    cycles arriving summed over the 8 XCDs."""
    from paper_1510_04895_amd import profile_summary as ps
    g = "void chebfd::(anonymous namespace)::k_gram<double>(...)"
    _write_pmc(tmp_path / "m", [(g, "SQ_INSTS_VALU_MFMA_MOPS_F64", 1000.0),
                                (g, "SQ_INSTS_VALU_MFMA_MOPS_F64", 3000.0),
                                (g, "SQ_VALU_MFMA_BUSY_CYCLES", 1024 * 50.0),
                                (g, "SQ_VALU_MFMA_BUSY_CYCLES", 1024 * 30.0),
                                (g, "GRBM_GUI_ACTIVE", 800.0), (g, "GRBM_GUI_ACTIVE", 800.0),
                                ("k_copy16(...)", "SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0)])
    monkeypatch.setattr(ps, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "profiles")
    out = ps.mfma(str(tmp_path / "m"), "mfma_test", "cmd")
    assert list(out) == ["k_gram<double>"]
    assert out["k_gram<double>"]["flops_per_dispatch"] == pytest.approx(2000 * 512)
    assert out["k_gram<double>"]["flops_max"] == pytest.approx(3000 * 512)
    assert out["k_gram<double>"]["mfma_busy_pct"] == pytest.approx(40.0)
    assert "| `k_gram<double>` | 2 |" in open(tmp_path / "profiles" / "mfma_test.md").read()
