"""Host logic of bench.py (no GPU): the multi-GPU refusal, the HBM-traffic
summary's scaling by the copy reference, and the per-launch-shape kernel
table of a rocprofv3 trace."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _write_counters(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_summary_scales_by_the_copy(tmp_path):
    # a 64^3 volume: the copy moves 4 * 64^3 bytes each way = 1024 KiB.
    # FETCH_SIZE reads half the copy's bytes (scale 2), WRITE_SIZE all of
    # them (scale 1); the sigma = 1 kernel then reads 1.5x and writes 1x of
    # its 4 B/voxel, so its traffic is (1.5 + 1) / 2 of the algorithmic 8 B.
    size = 64
    copy_kib = 4.0 * size ** 3 / 1024.0
    k1 = "void harpia::gauss_detail::gauss_fused_kernel<float, float, 3, false, 0, 1>(...)"
    k3 = "void harpia::morph_detail::gray_kernel<float, 1, 3, true>(...)"
    kb = "void harpia::morph_detail::bits_kernel<unsigned char, 0, 1, true>(...)"
    fetch = [{"Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": "FETCH_SIZE", "Counter_Value": copy_kib / 2},
             {"Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": "FETCH_SIZE", "Counter_Value": 3.0},
             {"Kernel_Name": k1, "Counter_Name": "FETCH_SIZE", "Counter_Value": 0.75 * copy_kib},
             {"Kernel_Name": k1, "Counter_Name": "FETCH_SIZE", "Counter_Value": 0.75 * copy_kib},
             {"Kernel_Name": k3, "Counter_Name": "FETCH_SIZE", "Counter_Value": 0.5 * copy_kib},
             {"Kernel_Name": kb, "Counter_Name": "FETCH_SIZE", "Counter_Value": 0.125 * copy_kib}]
    write = [{"Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": "WRITE_SIZE", "Counter_Value": copy_kib},
             {"Kernel_Name": k1, "Counter_Name": "WRITE_SIZE", "Counter_Value": copy_kib},
             {"Kernel_Name": k1, "Counter_Name": "WRITE_SIZE", "Counter_Value": copy_kib},
             {"Kernel_Name": k3, "Counter_Name": "WRITE_SIZE", "Counter_Value": 2 * copy_kib},
             {"Kernel_Name": kb, "Counter_Name": "WRITE_SIZE", "Counter_Value": 0.5 * copy_kib}]
    _write_counters(str(tmp_path / "f"), fetch)
    _write_counters(str(tmp_path / "w"), write)
    out = bench.traffic_summary(str(tmp_path / "f"), str(tmp_path / "w"), size, ("cf", "cw"))
    json.dumps(out)  # serialisable as written to profiles/
    assert out["copy_ref"]["FETCH_SIZE"]["scale"] == pytest.approx(2.0)
    assert out["copy_ref"]["WRITE_SIZE"]["scale"] == pytest.approx(1.0)
    s1 = out["ops"]["gauss_s1"]
    assert s1["dispatches"] == 2
    assert s1["alg_bytes_per_launch"] == 8 * size ** 3
    assert s1["traffic_over_alg"] == pytest.approx(2.5 / 2.0)
    # erode + dilate: two outputs, 12 B/voxel of algorithmic bytes
    e3 = out["ops"]["erode_dilate_ball3"]
    assert e3["alg_bytes_per_launch"] == 12 * size ** 3
    assert e3["traffic_over_alg"] == pytest.approx((1.0 + 2.0) / 3.0)
    # binary u8 pair: 1 B read, 2 B written per voxel (3 B algorithmic);
    # the counters read 0.25 x 4 B and 0.5 x 4 B per voxel after scaling
    b1 = out["ops"]["bin_u8_box1"]
    assert b1["alg_bytes_per_launch"] == 3 * size ** 3
    assert b1["traffic_over_alg"] == pytest.approx((1.0 + 2.0) / 3.0)
    # ops without both counters are left out
    assert "gauss_s4" not in out["ops"]


def test_traffic_summary_needs_the_copy(tmp_path):
    _write_counters(str(tmp_path / "f"), [{"Kernel_Name": "k", "Counter_Name": "FETCH_SIZE", "Counter_Value": 1}])
    _write_counters(str(tmp_path / "w"), [{"Kernel_Name": "k", "Counter_Name": "WRITE_SIZE", "Counter_Value": 1}])
    with pytest.raises(SystemExit):
        bench.traffic_summary(str(tmp_path / "f"), str(tmp_path / "w"), 64, ("cf", "cw"))


def test_stats_summary_groups_by_launch_shape(tmp_path):
    d = tmp_path / "t"
    d.mkdir()
    trace = [("void harpia::gauss_detail::gauss_fused_kernel<float, float, 3, false, 0, 1>(a)", 262144, 1024,
              0, 1000000),
             ("void harpia::gauss_detail::gauss_fused_kernel<float, float, 3, false, 0, 1>(a)", 262144, 1024,
              0, 3000000),
             ("void harpia::gauss_detail::gauss_fused_kernel<float, float, 3, false, 0, 1>(a)", 4096, 1024,
              0, 500000),
             ("at::native::other_kernel(x)", 1024, 256, 0, 100)]
    with open(d / "run_kernel_trace.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z", "Workgroup_Size_X",
                    "Workgroup_Size_Y", "Workgroup_Size_Z", "Start_Timestamp", "End_Timestamp"])
        for name, grid, wg, t0, t1 in trace:
            w.writerow([name, grid, 1, 1, wg, 1, 1, t0, t1])
    with open(d / "run_kernel_stats.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Name", "Calls", "AverageNs", "MinNs", "MaxNs", "TotalDurationNs", "Percentage"])
        w.writerow(["gauss_fused_kernel", 3, 1500000, 500000, 3000000, 4500000, 99.9])
    md = bench.stats_summary(str(d), "python3 bench.py", "title")
    lines = [l for l in md.splitlines() if l.startswith("| harpia::gauss_detail::gauss_fused_kernel")]
    # two launch shapes of the same kernel stay apart: 2 calls of 2000 us, 1 of 500 us
    assert len(lines) == 2
    big = [l for l in lines if "| 262144 |" in l][0]
    cells = [c.strip() for c in big.split("|")]
    assert cells[4] == "2" and float(cells[5]) == pytest.approx(2000.0)
    assert not any("other_kernel" in l for l in lines)
