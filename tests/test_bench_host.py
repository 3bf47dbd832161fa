"""Host logic of bench.py (CPU only): traffic summaries written from rocprofv3
CSV output and their calibration by a plain copy, the check that a traffic
record belongs to the current kernel sources, the roofline's choice of the
dominant kernel, and the refusal of more than one GPU."""
from __future__ import annotations

import csv
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _write(path, fields, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def _counters(path, counter, copy_kib, kernel_kib):
    rows = [{"Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": counter, "Counter_Value": copy_kib},
            {"Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": counter, "Counter_Value": 1.0}]
    rows += [{"Kernel_Name": "void rfim::k_fused_u8<true>(rfim::DevBeam const*, int)", "Counter_Name": counter,
              "Counter_Value": v} for v in kernel_kib]
    rows.append({"Kernel_Name": "rfim::k_zero_u64(unsigned long long*, long)", "Counter_Name": counter,
                 "Counter_Value": 7.0})
    _write(path, ["Kernel_Name", "Counter_Name", "Counter_Value"], rows)


def test_summarize_scales_counters_by_the_copy(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path / "profiles"))
    stats = tmp_path / "stats.csv"
    _write(stats, ["Name", "Calls", "AverageNs", "MinNs", "MaxNs", "Percentage"],
           [{"Name": "void rfim::k_fused_u8<true>(rfim::DevBeam const*, int)", "Calls": 12,
             "AverageNs": 900000, "MinNs": 880000, "MaxNs": 950000, "Percentage": 58.7}])
    fetch, write = tmp_path / "fetch.csv", tmp_path / "write.csv"
    copy_bytes = 1024000
    # the copy's FETCH_SIZE reads half its size (factor 2), its WRITE_SIZE all of it (factor 1)
    _counters(fetch, "FETCH_SIZE", copy_bytes / 1024 / 2, [1000.0, 1200.0])
    _counters(write, "WRITE_SIZE", copy_bytes / 1024, [2000.0, 2000.0])
    bench.summarize(str(stats), str(fetch), str(write), "the command", "wl", copy_bytes)

    md = open(tmp_path / "profiles" / "kernel_stats_wl.md").read()
    assert "the command" in md and "k_fused_u8" in md and "0.9000" in md
    kv = {}
    for line in open(tmp_path / "profiles" / "traffic_k_fused_u8_wl.txt"):
        if "=" in line and not line.startswith("#"):
            a, b = line.split("=", 1)
            kv[a.strip()] = b.strip()
    assert kv["src_hash"] == bench.source_hash("k_fused_u8")
    assert int(kv["read_bytes_per_launch"]) == 1100 * 1024 * 2
    assert int(kv["write_bytes_per_launch"]) == 2000 * 1024
    assert bench.read_traffic("k_fused_u8", "wl") == 1100 * 1024 * 2 + 2000 * 1024
    assert not os.path.exists(tmp_path / "profiles" / "traffic_k_zero_u64_wl.txt")


def test_traffic_of_other_sources_is_not_reported(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    with open(tmp_path / "traffic_k_fused_u8_wl.txt", "w") as f:
        f.write("kernel = k_fused_u8\nsrc_hash = 0000000000000000\ntraffic_bytes_per_launch = 123\n")
    assert bench.read_traffic("k_fused_u8", "wl") is None
    assert bench.read_traffic("k_td_rows_u8", "wl") is None   # no record at all


def test_source_hash_follows_the_kernel_group():
    assert bench.source_hash("k_fused_u8") == bench.source_hash("k_td_rows_u8")
    assert bench.source_hash("k_fused_f32") == bench.source_hash("k_td_rows_f32")
    assert bench.source_hash("k_fused_u8") != bench.source_hash("k_fused_f32")


def test_roofline_takes_the_kernel_with_the_most_time():
    kernels = {
        "k_td_rows_u8": {"launches": 10, "avg_ms": 0.6, "algo_bytes": 768, "gbs": 1280.0},
        "k_fused_u8": {"launches": 10, "avg_ms": 0.9, "algo_bytes": 1536, "gbs": 1706.7},
        "k_td_wide_f32": {"launches": 10, "avg_ms": 5.0, "algo_bytes": None, "gbs": None},
    }
    r = bench.roofline_of(kernels, "no-such-workload")
    assert r["kernel"] == "k_fused_u8"
    assert r["peak"] == 8000.0 and r["unit"] == "GB/s" and r["bound"] == "hbm"
    assert abs(r["frac"] - 1706.7 / 8000.0) < 1e-4
    assert r["traffic"] is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
