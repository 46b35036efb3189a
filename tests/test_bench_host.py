"""Host-only parts of bench.py (no GPU): the refusal of more than one GPU, and
the rocprofv3 CSV summaries that the committed profiles are made from.

The traffic summary scales each counter by the copy kernel of the same run
(known bytes / what the counter reads for it): synthetic counter files with a
known copy reading and a known kernel reading must give the bytes worked out
by hand here, per dispatch and summed over the counter's dimensions. The
counter summary's clock, matrix-core busy share and wave-wait shares are
checked the same way."""

import csv
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=300)


def test_more_than_one_gpu_is_refused():
    r = _bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def _write_counters(path, counter, rows):
    """rows: (kernel, dispatch, [values over dimensions], start_ns, end_ns)"""
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value",
                                           "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for kern, disp, values, t0, t1 in rows:
            for v in values:
                w.writerow({"Dispatch_Id": disp, "Kernel_Name": kern, "Counter_Name": counter,
                            "Counter_Value": v, "Start_Timestamp": t0, "End_Timestamp": t1})


def _kv(text):
    out = {}
    for line in text.splitlines():
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            out[k.strip()] = v.strip()
    return out


def test_traffic_summary_scales_by_the_copy_kernel(tmp_path):
    copy_bytes = 1 << 20
    # the copy reads 2048 KiB on FETCH_SIZE (split over two dimensions): scale 0.5
    # and 1024 KiB on WRITE_SIZE: scale 1.0
    k = "void k_gate<1, 5, 1, true>(KGate)"
    _write_counters(str(tmp_path / "f" / "a_counter_collection.csv"), "FETCH_SIZE", [
        ("k_copy(float2*, float2 const*, unsigned long)", 9, [1500.0, 548.0], 0, 1000),
        (k, 1, [3000.0, 1000.0], 0, 2000),          # 4000 KiB -> 2000 KiB read
        (k, 2, [2000.0], 0, 2000),                  # 2000 KiB -> 1000 KiB read
        ("other_kernel", 3, [99999.0], 0, 10),
    ])
    _write_counters(str(tmp_path / "w" / "a_counter_collection.csv"), "WRITE_SIZE", [
        ("k_copy(float2*, float2 const*, unsigned long)", 9, [1024.0], 0, 1000),
        (k, 1, [1200.0], 0, 2000),
        (k, 2, [1600.0], 0, 2000),
    ])
    r = _bench("--summarize", "traffic", str(tmp_path / "f"), str(tmp_path / "w"), r"k_gate<1, 5",
               str(copy_bytes), str(3 << 20))
    assert r.returncode == 0, r.stderr
    kv = _kv(r.stdout)
    assert float(kv["fetch_scale"]) == 0.5 and float(kv["write_scale"]) == 1.0
    assert kv["kernel dispatches (fetch run, write run)"] == "2, 2"
    read = (4000 + 2000) / 2 * 1024 * 0.5          # mean KiB x 1024 x scale
    write = (1200 + 1600) / 2 * 1024 * 1.0
    assert float(kv["read_bytes_per_launch"]) == read
    assert float(kv["write_bytes_per_launch"]) == write
    assert float(kv["traffic_bytes_per_launch"]) == read + write
    assert abs(float(kv["traffic_over_alg"]) - (read + write) / (3 << 20)) < 1e-4


def test_stats_summary_lists_every_kernel(tmp_path):
    d = tmp_path / "s"
    d.mkdir()
    with open(d / "x_kernel_stats.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage",
                                           "MinNs", "MaxNs"])
        w.writeheader()
        w.writerow({"Name": "kA", "Calls": 4, "TotalDurationNs": 10_000_000, "AverageNs": 2_500_000,
                    "Percentage": 80.0, "MinNs": 2_400_000, "MaxNs": 2_600_000})
        w.writerow({"Name": "kB", "Calls": 1, "TotalDurationNs": 2_500_000, "AverageNs": 2_500_000,
                    "Percentage": 20.0, "MinNs": 2_500_000, "MaxNs": 2_500_000})
    r = _bench("--summarize", "stats", str(d))
    assert r.returncode == 0, r.stderr
    lines = [ln.split() for ln in r.stdout.splitlines() if ln.strip().endswith(("kA", "kB"))]
    assert lines[0] == ["4", "2500.0", "2400.0", "2600.0", "10.00", "80.00", "kA"]
    assert lines[1] == ["1", "2500.0", "2500.0", "2500.0", "2.50", "20.00", "kB"]


def test_counters_summary_clock_and_shares(tmp_path):
    """Three dispatches of one kernel, 2 ms each (one slower dispatch moves
    no median): clock = GRBM_GUI_ACTIVE / 8 XCDs / duration, matrix-core
    busy share = busy cycles / (1024 SIMDs x clock cycles), wait shares =
    SQ_WAIT_ANY and SQ_WAIT_INST_ANY over SQ_WAVE_CYCLES."""
    k = "void k_fused_wide<1>(KFusedWide)"
    rows = []
    for disp, dur_ns, scale in ((1, 2_000_000, 1.0), (2, 2_000_000, 1.0), (3, 3_000_000, 1.5)):
        cycles = 2.2e9 * dur_ns / 1e9                     # 2.2 GHz
        vals = {"GRBM_GUI_ACTIVE": [8 * cycles],
                "SQ_VALU_MFMA_BUSY_CYCLES": [0.25 * 1024 * cycles, 0.25 * 1024 * cycles],
                "SQ_WAVE_CYCLES": [1e9 * scale], "SQ_WAIT_ANY": [7.5e8 * scale],
                "SQ_WAIT_INST_ANY": [1e8 * scale]}
        for ctr, vs in vals.items():
            rows.append((ctr, disp, vs, dur_ns))
    path = tmp_path / "c" / "x_counter_collection.csv"
    path.parent.mkdir()
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value",
                                           "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for ctr, disp, vs, dur_ns in rows:
            for v in vs:
                w.writerow({"Dispatch_Id": disp, "Kernel_Name": k, "Counter_Name": ctr, "Counter_Value": v,
                            "Start_Timestamp": 10, "End_Timestamp": 10 + dur_ns})
    r = _bench("--summarize", "counters", str(tmp_path / "c"))
    assert r.returncode == 0, r.stderr
    out = r.stdout
    assert "dispatches 3, median duration 2.0000 ms" in out
    assert "clock GHz (GRBM_GUI_ACTIVE / 8 XCDs / duration): 2.20" in out
    assert "MFMA busy share at that clock (busy / (1024 SIMDs x cycles)): 0.500" in out
    assert "(SQ_WAIT_ANY / SQ_WAVE_CYCLES): 0.750" in out
    assert "(SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES): 0.100" in out
