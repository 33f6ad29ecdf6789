"""Host-side measurement logic (no GPU): the per-kernel algorithmic byte and
flop counts, the roofline record's choice of kernel, the counter summaries
and the staleness rule of the measured-traffic records."""
import csv
import json
import os

import pytest

import bench
from paper_2607_02335_amd import profiling


def test_kernel_bytes_match_their_definitions():
    p, n = 3, 64
    cell = n ** 3 * (p + 1) ** 3 * 8
    uniq = (n * p + 1) ** 3 * 8
    patch = (n - 1) ** 3 * (2 * p - 1) ** 3 * 8
    # every phase of an operation is charged the operation's bytes: read one
    # cell-wise vector, write one (16 B per cell DoF in FP64)
    for lab in ("apply", "pi_assemble", "pi_solve", "pi_combine", "pi_sweep"):
        assert bench.kernel_bytes(lab, p, n) == 2 * cell == 268435456
    assert bench.kernel_bytes("unknown", p, n) is None
    # the design floors: the arrays each kernel has to touch once
    assert bench.design_bytes("pi_assemble", p, n) == cell + uniq
    assert bench.design_bytes("pi_solve", p, n) == uniq + patch
    assert bench.design_bytes("pi_combine", p, n) == patch + cell
    assert bench.design_bytes("pi_sweep", p, n) == uniq + cell          # reads the assembled residual
    # FP32 storage
    assert bench.kernel_bytes("apply", 7, 24, 4, 4) == 2 * 24 ** 3 * 512 * 4
    # structured DSS: both copies of every face pair, read and written, per axis pass
    assert bench.op_bytes("dss", 1, 2, 8) == 4 * 8 * 4 * 3 * 1 * 2 * 2


def test_apply_flops_follow_the_papers_laplace_table():
    """14(p+1) useful flops per cell DoF: the paper's table lists theory
    TFLOP/s beside cell-wise GDoF/s, whose quotient is the per-DoF count
    (p >= 3; p = 1, 2 use an even-odd factorisation with fewer)."""
    rows = [l.split() for l in open(os.path.join(os.path.dirname(__file__), "golden", "laplace_table.txt"))
            if l.strip() and not l.startswith("#")]
    for deg, cell_gdofs, _, _, theory_tf in rows:
        p = int(deg)
        per_dof = float(theory_tf) * 1e12 / (float(cell_gdofs) * 1e9)
        if p >= 3:
            assert abs(bench.op_flops("apply", p, 1) / (p + 1) ** 3 - per_dof) / per_dof < 0.002, p
        else:
            assert bench.op_flops("apply", p, 1) / (p + 1) ** 3 >= per_dof


def test_kernel_flops():
    # Q3 patch: 12 nP^4 + nP^3 with nP = 5 -> 7625 per patch
    assert bench.kernel_flops("pi_solve", 3, 2) == 7625
    assert bench.kernel_flops("pi_sweep", 3, 2) == 7625
    assert bench.kernel_flops("pi_combine", 3, 2) is None
    assert bench.kernel_flops("apply", 7, 1) == 512 * 14 * 8


def test_roofline_picks_the_largest_share():
    rec = dict(p=3, n=64, kernels=[
        dict(label="apply", p=3, prec=0, launches=20, total_ms=1.1, avg_us=55.0),
        dict(label="pi_assemble", p=3, prec=0, launches=20, total_ms=0.6, avg_us=30.0),
        dict(label="pi_solve", p=3, prec=0, launches=20, total_ms=2.9, avg_us=145.0),
        dict(label="pi_combine", p=3, prec=0, launches=20, total_ms=2.3, avg_us=115.0),
        dict(label="dot", p=3, prec=0, launches=20, total_ms=9.0, avg_us=450.0)])   # no byte model: ignored
    r = bench.roofline(rec, workload="no_such_workload", copy_gbs=6000.0)
    assert r["kernel"] == "pi_solve" and r["op"] == "patch_inverse" and r["traffic"] is None
    assert r["achieved"] == pytest.approx(bench.kernel_bytes("pi_solve", 3, 64) / 145e-6 / 1e9, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"], rel=1e-3)
    assert r["frac_of_copy_peak"] == pytest.approx(r["achieved"] / 6000.0, rel=1e-3)
    # the patch inverse as one unit: its three phases' times summed
    pi = r["ops"]["patch_inverse"]
    assert pi["time_us"] == pytest.approx(290.0)
    assert pi["GB/s"] == pytest.approx(2 * 64 ** 3 * 64 * 8 / 290e-6 / 1e9, rel=1e-3)
    assert pi["flop_frac"] == pytest.approx(63 ** 3 * 7625 / 290e-6 / 1e12 / 78.6, rel=1e-3)
    assert r["ops"]["apply"]["hbm_frac"] == pytest.approx(2 * 64 ** 3 * 64 * 8 / 55e-6 / 1e9 / 8000, rel=1e-3)


def _write_counters(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_traffic_summary_scales_by_the_copy_calibration(tmp_path):
    k = "void fem::k_pi_solve_g<3, double, 32, false>(fem::LaunchTable)"
    copy = "__amd_rocclr_copyBuffer"
    _write_counters(tmp_path / "f", [dict(Kernel_Name=k, Counter_Name="FETCH_SIZE", Counter_Value=100.0)] * 3)
    _write_counters(tmp_path / "w", [dict(Kernel_Name=k, Counter_Name="WRITE_SIZE", Counter_Value=400.0)])
    # the copy of 1 MiB reads as 512 KiB fetched and 1024 KiB written
    _write_counters(tmp_path / "cf", [dict(Kernel_Name=copy, Counter_Name="FETCH_SIZE", Counter_Value=512.0)])
    _write_counters(tmp_path / "cw", [dict(Kernel_Name=copy, Counter_Name="WRITE_SIZE", Counter_Value=1024.0)])
    out = tmp_path / "traffic_x.md"
    profiling.main(["traffic", "--workload", "x", "--command", "c", "--fetch", str(tmp_path / "f"),
                    "--write", str(tmp_path / "w"), "--calib-fetch", str(tmp_path / "cf"),
                    "--calib-write", str(tmp_path / "cw"), "--calib-bytes", str(1 << 20), "-o", str(out)])
    rec = json.load(open(tmp_path / "traffic_x.json"))
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    kk = rec["kernels"]["pi_solve"]
    assert kk["read_bytes"] == pytest.approx(100 * 1024 * 2.0)
    assert kk["write_bytes"] == pytest.approx(400 * 1024 * 1.0)
    assert rec["sources_sha256"] == profiling.sources_hash()
    assert "k_pi_solve_g" in open(out).read()


def test_measured_traffic_is_dropped_when_sources_change(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = {"sources_sha256": profiling.sources_hash(), "kernels": {"pi_solve": {"bytes": 1234.4}}}
    (prof / "traffic_w.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("w", "pi_solve") == 1234
    assert bench.measured_traffic("w", "apply") is None
    rec["sources_sha256"] = "0" * 64
    (prof / "traffic_w.json").write_text(json.dumps(rec))
    assert bench.measured_traffic("w", "pi_solve") is None


def test_stats_and_counters_summaries(tmp_path):
    stats = tmp_path / "s.csv"
    with open(stats, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"])
        w.writerow(["void fem::k_apply_reg<3, double, 0, false>(x)", 10, 500000, 50000, 40.0, 49000, 52000, 1.0])
    out = tmp_path / "k.md"
    profiling.main(["stats", str(stats), "--workload", "w", "--command", "c", "-o", str(out)])
    text = open(out).read()
    assert "k_apply_reg<3, double, 0, false>" in text and "| apply |" in text and "50.0" in text
    _write_counters(tmp_path / "a", [dict(Kernel_Name="void fem::k_pi_solve_mfma<7>(x)", Counter_Name="MfmaUtil",
                                          Counter_Value=v) for v in (30.0, 40.0)])
    out2 = tmp_path / "c.md"
    profiling.main(["counters", str(tmp_path / "a"), "--workload", "w", "--command", "c", "-o", str(out2)])
    assert "| `k_pi_solve_mfma<7>` | 35.0 |" in open(out2).read()
