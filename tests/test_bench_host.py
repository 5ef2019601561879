"""Host-side logic of bench.py and the profile summariser (no GPU).

Pins: the multi-GPU request exits before touching a device with the
one-GPU message; the algorithmic byte count of a plan-update launch and
the exponential count of the assignment against hand counts on a tiny
workload; the committed traffic summary is used only for the kernel source
it was taken on; the counter calibration scales by the copy probe."""
import csv
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1510_00012_amd import profiling  # noqa: E402


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"),
                        "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def _tiny():
    # three instances with 2, 3 and 1 support points in d = 3
    off = np.array([0, 2, 5, 6], dtype=np.int64)
    return {"offsets": off, "X": np.zeros((6, 3)), "W": np.ones(6)}


def test_algorithmic_bytes_hand_count():
    wl = _tiny()
    m, esz = 4, 4
    E = m * 6  # plan entries
    # Pi1 and Lambda read + written, support coordinates and weights, per
    # instance two offsets (int64) and one work-list entry (int32)
    want = 4 * E * esz + 6 * 3 * esz + 6 * esz + 3 * (8 + 8 + 4)
    assert bench.algorithmic_bytes("iter_ba", wl, m, esz) == want
    # d > 4: one cached cost entry per plan entry instead of coordinates
    wl5 = dict(wl, X=np.zeros((6, 5)))
    want5 = 4 * E * esz + E * esz + 6 * esz + 3 * 20
    assert bench.algorithmic_bytes("iter_ba", wl5, m, esz) == want5


def test_assignment_exponential_count():
    wl = _tiny()
    # K centroids of m points, 6 instance points in all, 2 exponentials per
    # entry and iteration, for the surviving fraction of pairs
    assert bench.assign_exps(wl, 5, 4, 100) == 2 * 5 * 4 * 6 * 100
    assert bench.assign_exps(wl, 5, 4, 100, 0.25) == 2 * 5 * 4 * 6 * 100 / 4


def test_traffic_summary_is_tied_to_the_kernel_source():
    h = bench.kernel_source_hash()
    assert h == profiling.kernel_source_hash()
    path = os.path.join(ROOT, "profiles", "traffic_k_iter_ba_gmm_d3_n65536_k16.json")
    rec = json.load(open(path))
    got = bench.load_traffic("k_iter_ba", "gmm_d3_n65536_k16", h)
    if rec["kernel_source_hash"] == h:
        assert got == rec["hbm_bytes_per_launch"]
    else:
        assert got is None
    assert bench.load_traffic("k_iter_ba", "gmm_d3_n65536_k16", "0" * 16) is None
    assert bench.load_traffic("k_iter_ba", "no_such_workload", h) is None


def test_counter_calibration(tmp_path):
    # a copy probe of 4 MiB whose FETCH_SIZE reads half its size, a kernel
    # with two dispatches
    def write(path, counter, rows):
        with open(path, "w", newline="") as f:
            w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name",
                                              "Counter_Value"])
            w.writeheader()
            for name, v in rows:
                w.writerow({"Kernel_Name": name, "Counter_Name": counter,
                            "Counter_Value": v})
    fcsv, wcsv = tmp_path / "f.csv", tmp_path / "w.csv"
    write(fcsv, "FETCH_SIZE", [("__amd_rocclr_copyBuffer", 2048.0),
                               ("__amd_rocclr_copyBuffer", 3.0),
                               ("k_iter_ba<float>", 100.0),
                               ("k_iter_ba<float>", 300.0),
                               ("k_assign", 1e6)])
    write(wcsv, "WRITE_SIZE", [("__amd_rocclr_copyBuffer", 4096.0),
                               ("k_iter_ba<float>", 50.0),
                               ("k_iter_ba<float>", 150.0)])
    rec = profiling.traffic(str(fcsv), str(wcsv), "k_iter_ba", "tiny", 4,
                            str(tmp_path / "t.json"), "cmd")
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0
    # mean raw per dispatch 200 KiB read (x2) and 100 KiB written
    assert rec["hbm_bytes_per_launch"] == (200.0 * 2.0 + 100.0) * 1024.0
    # the library's copy probe takes precedence (median of its dispatches);
    # two bucket dispatches per timed launch double the bytes per launch
    write(fcsv, "FETCH_SIZE", [("__amd_rocclr_copyBuffer", 2048.0),
                               ("k_copy_probe(float4*)", 4096.0),
                               ("k_copy_probe(float4*)", 4000.0),
                               ("k_copy_probe(float4*)", 4100.0),
                               ("k_iter_ba<float>", 100.0),
                               ("k_iter_ba<float>", 300.0)])
    write(wcsv, "WRITE_SIZE", [("k_copy_probe(float4*)", 8192.0),
                               ("k_iter_ba<float>", 50.0),
                               ("k_iter_ba<float>", 150.0)])
    rec = profiling.traffic(str(fcsv), str(wcsv), "k_iter_ba", "tiny", 8,
                            str(tmp_path / "t.json"), "cmd", 2)
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0
    assert rec["hbm_bytes_per_launch"] == 2 * (200.0 * 2.0 + 100.0) * 1024.0


def test_traffic_adds_the_passes_beside_the_plan_update(tmp_path):
    """Matrix-core passes launched within some iterations add their bytes
    to those iterations; the plan-update dispatches count the iterations."""
    def write(path, counter, rows):
        with open(path, "w", newline="") as f:
            w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name",
                                              "Counter_Value"])
            w.writeheader()
            for name, v in rows:
                w.writerow({"Kernel_Name": name, "Counter_Name": counter,
                            "Counter_Value": v})
    fcsv, wcsv = tmp_path / "f.csv", tmp_path / "w.csv"
    # 4 iterations of one dispatch each, one k_sup_mfma and one k_cost_mfma
    write(fcsv, "FETCH_SIZE", [("k_copy_probe(float4*)", 2048.0)] +
          [("k_iter_ba<float>", 100.0)] * 4 +
          [("k_sup_mfma<32>", 40.0), ("k_cost_mfma<8>", 20.0)])
    write(wcsv, "WRITE_SIZE", [("k_copy_probe(float4*)", 4096.0)] +
          [("k_iter_ba<float>", 50.0)] * 4 + [("k_cost_mfma<8>", 8.0)])
    rec = profiling.traffic(str(fcsv), str(wcsv),
                            "k_iter_ba,k_sup_mfma,k_cost_mfma", "tiny", 4,
                            str(tmp_path / "t.json"), "cmd")
    assert rec["kernel"] == "k_iter_ba"
    reads = (400.0 + 60.0) / 4 * 2.0
    writes = (200.0 + 8.0) / 4
    assert rec["hbm_bytes_per_launch"] == (reads + writes) * 1024.0
