"""CPU checks of the benchmark's host logic: it refuses more than one GPU, prices kernels
with the stated algorithmic bytes, and turns two counter runs into copy-calibrated HBM
bytes per launch (tied to the current sources)."""

import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_algorithmic_bytes_of_the_10m_edge_workload():
    E, N, K, M = 10_000_000, 600_000, 50, 20_000_000
    # bucket_embed: (row-in-bucket u16, col, w) per entry, {c, y} and s per node, Z once
    assert bench.algorithmic_bytes("bucket_embed", E, N, K, M, True, 0) == 10 * M + 12 * N + 4 * N * K == 327_200_000
    assert bench.algorithmic_bytes("bucket_embed", E, N, K, M, False, 0) == 6 * M + 12 * N + 4 * N * K
    assert bench.algorithmic_bytes("a_hist", E, N, K, M, True, 0) == 8 * E + 4 * N
    assert bench.algorithmic_bytes("edge_scatter", E, N, K, M, True, 0) == 12 * E + 8 * N + 4 * N * K
    assert bench.algorithmic_bytes("no_such_kernel", E, N, K, M, True, 0) == 0


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (name, v) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": v})


def test_traffic_calibration(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path / "profiles"))
    gib_kib = (1 << 30) / 1024.0
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    # the counter reads half of the copied bytes on fetch, all of them on write
    _counter_csv(fetch, "FETCH_SIZE", [("__amd_rocclr_copyBuffer", gib_kib / 2),
                                       ("void gee::bucket_embed<unsigned short, true>(...)", 1000.0),
                                       ("void gee::bucket_embed<unsigned short, true>(...)", 3000.0),
                                       ("gee::bucket_embed_fix(...)", 99999.0)])
    _counter_csv(write, "WRITE_SIZE", [("__amd_rocclr_copyBuffer", gib_kib),
                                       ("void gee::bucket_embed<unsigned short, true>(...)", 500.0),
                                       ("void gee::bucket_embed<unsigned short, true>(...)", 500.0)])
    path = bench.write_traffic(str(fetch), str(write), "bucket_embed", "wl", "cmd")
    assert path.startswith(str(tmp_path))
    d = bench.read_traffic("bucket_embed", "wl")
    assert d["fetch_launches"] == 2 and d["write_launches"] == 2  # bucket_embed_fix is another kernel
    assert d["fetch_calibration_factor"] == pytest.approx(2.0)
    assert d["fetch_bytes_per_launch"] == 2000 * 1024 * 2
    assert d["write_bytes_per_launch"] == 500 * 1024
    assert d["bytes_per_launch"] == d["fetch_bytes_per_launch"] + d["write_bytes_per_launch"]
    # figures taken from other sources do not count
    monkeypatch.setattr(bench, "source_hash", lambda: "0000000000000000")
    assert bench.read_traffic("bucket_embed", "wl") is None


def test_committed_traffic_is_at_least_the_algorithmic_bytes():
    d = bench.read_traffic("bucket_embed", "chunglu_n600k_e10m_k50")
    if d is None:
        pytest.skip("the committed counter summary was taken from other HIP sources")
    assert d["bytes_per_launch"] > bench.algorithmic_bytes("bucket_embed", 10_000_000, 600_000, 50, 20_000_000,
                                                            True, 0)
