"""Host logic of bench.py's profile summaries, on synthetic counter files:
copy-calibrated HBM traffic, issued FP64 operations, and the rule that a
committed summary is used only for the tracker variant and library sources
it was taken on."""
import csv
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def write_counters(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "p_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for k, c, v in rows:
            w.writerow({"Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})


KNAME = "void gm::%s(gm::TArgs)" % bench.TRACK_KERNEL


@pytest.fixture(autouse=True)
def _summaries_to_tmp(tmp_path, monkeypatch):
    """No test here writes a committed profile summary: every summary path
    points into the test's own directory."""
    monkeypatch.setattr(bench, "TRAFFIC_JSON", str(tmp_path / "k_traffic.json"))
    monkeypatch.setattr(bench, "ISSUE_JSON", str(tmp_path / "k_fp64_issue.json"))
    monkeypatch.setattr(bench, "TRACE_TXT", str(tmp_path / "k_kernel_trace.txt"))
    monkeypatch.setattr(bench, "SUMMARY_TARGETS", {k: dict(v, prefix=str(tmp_path / k))
                                                   for k, v in bench.SUMMARY_TARGETS.items()})


def test_traffic_is_scaled_by_the_copy(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_JSON", str(tmp_path / "traffic.json"))
    f, w = str(tmp_path / "f"), str(tmp_path / "w")
    # a 1 MiB copy reads 1024 KiB and writes 1024 KiB; the counters report half and all of it
    write_counters(f, [("__amd_rocclr_copyBuffer", "FETCH_SIZE", 512.0), (KNAME, "FETCH_SIZE", 100.0),
                       (KNAME, "FETCH_SIZE", 300.0), ("other", "FETCH_SIZE", 1e9)])
    write_counters(w, [("__amd_rocclr_copyBuffer", "WRITE_SIZE", 1024.0), (KNAME, "WRITE_SIZE", 50.0),
                       (KNAME, "WRITE_SIZE", 150.0)])
    bench.summarize_traffic(f, w, ["cmd"], copy_mib=1)
    d = json.load(open(bench.TRAFFIC_JSON))
    assert d["launches"] == 2 and d["kernel"] == bench.TRACK_KERNEL
    assert d["copy_calibration"]["fetch_factor"] == pytest.approx(2.0)
    assert d["copy_calibration"]["write_factor"] == pytest.approx(1.0)
    assert d["bytes_per_launch"] == pytest.approx(1024 * (200.0 * 2.0 + 100.0 * 1.0))
    assert bench.measured_traffic(bench.TRACK_KERNEL) == pytest.approx(d["bytes_per_launch"])
    assert bench.measured_traffic(bench.track_variant(2, 64)) is None       # another variant
    d["kernel_source_hash"] = "0" * 16
    json.dump(d, open(bench.TRAFFIC_JSON, "w"))
    assert bench.measured_traffic(bench.TRACK_KERNEL) is None               # other sources


def test_issued_fp64_convention(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ISSUE_JSON", str(tmp_path / "issue.json"))
    d = str(tmp_path / "i")
    rows = []
    for v in (1.0, 3.0):       # two launches: per-launch means 2, 4, 6, 8
        rows += [(KNAME, "SQ_INSTS_VALU_ADD_F64", v), (KNAME, "SQ_INSTS_VALU_MUL_F64", 2 * v),
                 (KNAME, "SQ_INSTS_VALU_TRANS_F64", 3 * v), (KNAME, "SQ_INSTS_VALU_FMA_F64", 4 * v),
                 (KNAME, "SQ_INSTS_VALU", 100 * v)]
    write_counters(d, rows)
    bench.summarize_issue(d, ["cmd"])
    out = json.load(open(bench.ISSUE_JSON))
    assert out["launches"] == 2
    assert out["issued_fp64_flop_per_launch"] == pytest.approx(64 * (2 + 4 + 6) + 128 * 8)
    assert bench.measured_issue(bench.TRACK_KERNEL) == pytest.approx(out["issued_fp64_flop_per_launch"])


def test_variant_names_match_the_compiled_kernels():
    assert bench.track_variant(2, 1) == "track_kernel_ks<2, false, false, true>"
    assert bench.track_variant(2, 4, const_bias=False) == "track_kernel_ks<2, false, true, false>"
    assert bench.track_variant(3, 64, kerr=False) == "track_kernel_flat<3, false, true>"


def test_kerr_flop_count_from_counters():
    """The tracker's algorithmic work from the event counters: every point
    (step or sub-step), corrector pass, split and load counted once."""
    st = [0] * 33
    st[bench.S["STEPS"]], st[bench.S["SCATTER"]], st[bench.S["VERLET_IT"]] = 1000, 10, 2500
    st[bench.S["ROOTS"]], st[bench.S["CHILDREN"]] = 7, 3
    P = bench.KS_FLOPS_PER
    assert bench.ks_flops(st) == P["point"] * 1010 + P["corrector"] * 2500 + P["split"] * 10 + P["load"] * 10


def test_flat_target_summary(tmp_path):
    """A summary of the flat tracker's counters takes that kernel's rows
    only and goes to the flat target's own file."""
    t = dict(bench.SUMMARY_TARGETS["scattering_sphere"], prefix=str(tmp_path / "flat"))
    kf = "void gm::%s(gm::TArgs)" % t["kernel"]
    d = str(tmp_path / "pmc")
    rows = []
    for k, v in ((kf, 1.0), (kf, 3.0), (KNAME, 100.0)):
        rows += [(k, "SQ_INSTS_VALU_ADD_F64", v), (k, "SQ_INSTS_VALU_MUL_F64", v),
                 (k, "SQ_INSTS_VALU_TRANS_F64", v), (k, "SQ_INSTS_VALU_FMA_F64", v), (k, "SQ_INSTS_VALU", v)]
    write_counters(d, rows)
    bench.summarize_issue(d, ["cmd"], t)
    out = json.load(open(str(tmp_path / "flat_fp64_issue.json")))
    assert out["kernel"] == t["kernel"] and out["launches"] == 2
    assert out["issued_fp64_flop_per_launch"] == pytest.approx(64 * 3 * 2.0 + 128 * 2.0)
