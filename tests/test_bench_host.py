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
    # bucket_embed: (column word with its row in bucket packed in, w) per entry, the 5-byte
    # {c, y} record and s per node, Z once
    assert bench.algorithmic_bytes("bucket_embed", E, N, K, M, True, 0) == 8 * M + 9 * N + 4 * N * K == 285_400_000
    assert bench.algorithmic_bytes("bucket_embed", E, N, K, M, False, 0) == 4 * M + 9 * N + 4 * N * K
    assert bench.algorithmic_bytes("a_hist", E, N, K, M, True, 0) == 8 * E + 4 * N
    assert bench.algorithmic_bytes("edge_scatter", E, N, K, M, True, 0) == 12 * E + 8 * N + 4 * N * K
    assert bench.algorithmic_bytes("no_such_kernel", E, N, K, M, True, 0) == 0


def test_step_bytes_follow_the_definitions():
    E, N, K, M = 10_000_000, 600_000, 50, 20_000_000
    # a4-a6 from a CSR: row_ptr + col + val + labels + gathered c + Z
    assert bench.step_bytes("a4_a6", E, N, K, M, True) == 4 * (N + 1) + 8 * M + 4 * N + 4 * N + 4 * N * K
    assert round(bench.step_bytes("a4_a6", E, N, K, M, True) / 1e6, 1) == 287.2
    # degrees: row_ptr + val in, s out; embed = degrees + a4-a6 (372 MB on this workload)
    assert round(bench.step_bytes("a3", E, N, K, M, True) / 1e6, 1) == 84.8
    assert round(bench.step_bytes("embed", E, N, K, M, True) / 1e6) == 372
    # the whole call's minimum: edge list + labels in, Z out
    assert bench.step_bytes("e2e", E, N, K, M, True) == 12 * E + 4 * N + 4 * N * K
    assert bench.step_bytes("e2e", E, N, K, M, False) == 8 * E + 4 * N + 4 * N * K
    assert bench.KERNEL_STEP["bucket_embed"] == "a4_a6" and bench.KERNEL_STEP["bucket_degree"] == "a3"


def _counter_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (disp, name, counter, v) in enumerate(rows):
            w.writerow({"Dispatch_Id": disp, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": v})


def test_traffic_from_request_counts(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path / "profiles"))
    a, b = tmp_path / "a.csv", tmp_path / "b.csv"
    emb = "void gee::bucket_embed<unsigned short, true>(gee::Batch, ...)"
    seg = "void gee::seg_scatter<unsigned short, false>(...)"
    rows_a, rows_b = [], []
    # a 1 GiB copy: 2^23 read requests of 128 bytes, 2^24 write requests of 64 bytes
    for c, v in (("TCC_EA0_RDREQ_32B_sum", 0), ("TCC_EA0_RDREQ_64B_sum", 0), ("TCC_EA0_RDREQ_128B_sum", 1 << 23),
                 ("TCC_EA0_RDREQ_sum", 1 << 23)):
        rows_a.append((1, "__amd_rocclr_copyBuffer", c, v))
    for c, v in (("TCC_EA0_WRREQ_sum", 1 << 24), ("TCC_EA0_WRREQ_64B_sum", 1 << 24),
                 ("TCC_EA0_RDREQ_DRAM_32B_sum", 1 << 25), ("TCC_EA0_WRREQ_WRITE_DRAM_32B_sum", 1 << 25)):
        rows_b.append((1, "__amd_rocclr_copyBuffer", c, v))
    # two launches of bucket_embed (per-launch means), one of pass B's segment scatter
    for disp, scale in ((2, 1), (3, 3)):
        for c, v in (("TCC_EA0_RDREQ_32B_sum", 10), ("TCC_EA0_RDREQ_64B_sum", 20), ("TCC_EA0_RDREQ_128B_sum", 30),
                     ("TCC_EA0_RDREQ_sum", 60)):
            rows_a.append((disp, emb, c, v * scale))
        for c, v in (("TCC_EA0_WRREQ_sum", 50), ("TCC_EA0_WRREQ_64B_sum", 40), ("TCC_EA0_RDREQ_DRAM_32B_sum", 7),
                     ("TCC_EA0_WRREQ_WRITE_DRAM_32B_sum", 9)):
            rows_b.append((disp, emb, c, v * scale))
    for c in ("TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_64B_sum", "TCC_EA0_RDREQ_128B_sum", "TCC_EA0_RDREQ_sum"):
        rows_a.append((4, seg, c, 1))
    for c in ("TCC_EA0_WRREQ_sum", "TCC_EA0_WRREQ_64B_sum", "TCC_EA0_RDREQ_DRAM_32B_sum",
              "TCC_EA0_WRREQ_WRITE_DRAM_32B_sum"):
        rows_b.append((4, seg, c, 1))
    _counter_csv(a, rows_a)
    _counter_csv(b, rows_b)
    path = bench.write_traffic(str(a), str(b), "wl", "cmd")
    assert path.startswith(str(tmp_path))
    d = bench.read_traffic("wl")
    assert d["copy_check"]["read_bytes"] == 1 << 30 and d["copy_check"]["write_bytes"] == 1 << 30
    k = d["kernels"]["bucket_embed"]
    assert k["launches"] == 2
    # means of the two launches: 20 x 32 + 40 x 64 + 60 x 128 read; 40 x 64 + 20 x 32 written
    assert k["read_bytes"] == 20 * 32 + 40 * 64 + 60 * 128
    assert k["write_bytes"] == 80 * 64 + 20 * 32
    assert k["bytes"] == k["read_bytes"] + k["write_bytes"]
    assert k["dram_read_bytes"] == 14 * 32 and k["dram_write_bytes"] == 18 * 32
    assert "b_scatter" in d["kernels"] and "seg_scatter" not in d["kernels"]
    # figures taken from other sources do not count
    monkeypatch.setattr(bench, "source_hash", lambda: "0000000000000000")
    assert bench.read_traffic("wl") is None


def test_kernel_names_map_to_the_hook_names():
    assert bench.kernel_key("void gee::a_scatter<unsigned short>(gee::Batch, long)") == "a_scatter"
    assert bench.kernel_key("void gee::seg_scatter<unsigned short, true>(...)") == "c_scatter"
    assert bench.kernel_key("gee::seg_hist(...)") == "b_hist"
    assert bench.kernel_key("__amd_rocclr_copyBuffer") == "copy"


def test_committed_traffic_is_at_least_the_algorithmic_bytes():
    d = bench.read_traffic("chunglu_n600k_e10m_k50")
    if d is None:
        pytest.skip("the committed counter summary was taken from other HIP sources")
    assert d["copy_check"]["read_bytes"] == pytest.approx(1 << 30, rel=0.01)
    emb = d["kernels"]["bucket_embed"]["bytes"]
    assert emb > bench.step_bytes("a4_a6", 10_000_000, 600_000, 50, 20_000_000, True)


def test_kernel_trace_summary(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path / "profiles"))
    p = tmp_path / "trace.csv"
    names = ["gee::a_hist(...)", "void gee::a_scatter<unsigned short>(...)", "gee::bucket_embed_fix(...)"]
    with open(p, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        t = 1000
        for call, durs in enumerate(([10_000, 50_000, 5_000], [12_000, 70_000, 5_000], [11_000, 60_000, 7_000])):
            for n, d in zip(names, durs):
                w.writerow({"Kernel_Name": n, "Start_Timestamp": t, "End_Timestamp": t + d})
                t += d + 500
            w.writerow({"Kernel_Name": "void at::native::fill(...)", "Start_Timestamp": t, "End_Timestamp": t + 9})
            t += 100_000
    path = bench.write_trace(str(p), "wl", "cmd")
    text = open(path).read()
    d = json.loads(text[text.index("```json") + 7:text.rindex("```")])
    assert d["calls"] == 3
    assert d["kernels_us"] == {"a_hist": 11.0, "a_scatter": 60.0, "bucket_embed_fix": 5.0}
    assert d["span_us"] == 79.0  # spans 66, 88 and 79 us
