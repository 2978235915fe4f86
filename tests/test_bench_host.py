"""Host-side logic of bench.py (no GPU): the counter digest that turns
rocprofv3 FETCH_SIZE / WRITE_SIZE rows into HBM bytes per launch, the
grouping of stage timings by kernel symbol, the per-kernel roofline, and
the refusal of more than one GPU."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        wr = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        wr.writeheader()
        for name, value in rows:
            wr.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_pmc_digest_scales_by_the_copy_kernel(tmp_path):
    # a 256 MiB copy reads back FETCH = half its bytes and WRITE = all of them
    copy = "__amd_rocclr_copyBuffer"
    kern = "void mlfma::(anonymous namespace)::k_translate_reg<2>(mlfma::(anonymous namespace)::TrLevels<float>, int)"
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    _counter_csv(f, "FETCH_SIZE", [(copy, 131072.0), (kern, 1000.0), (kern, 3000.0)])
    _counter_csv(w, "WRITE_SIZE", [(copy, 262144.0), (kern, 500.0), (kern, 500.0)])
    out = tmp_path / "digest.json"
    bench.pmc_digest(str(f), str(w), 256, str(out), "test")
    rec = json.loads(out.read_text())
    assert rec["calibration"]["fetch_scale"] == pytest.approx(2.0)
    assert rec["calibration"]["write_scale"] == pytest.approx(1.0)
    k = rec["kernels"]["k_translate_reg<2>"]
    assert k["dispatches"] == 2
    assert k["fetch_bytes_per_launch"] == pytest.approx(2000.0 * 1024 * 2.0)
    assert k["write_bytes_per_launch"] == pytest.approx(500.0 * 1024)
    assert rec["source_sha256"] == bench.source_digest()


def test_kernel_table_groups_by_recorded_symbol_and_rooflines():
    stages = [
        {"name": "aggregate_l1", "kernel": "k_agg_stream<float, 6, 32>", "total_ms": 2.0, "launches": 1,
         "bytes_per_launch": 4e9, "flops_per_launch": 0.0},
        {"name": "aggregate_l2", "kernel": "k_agg_stream<float, 6, 32>", "total_ms": 1.0, "launches": 1,
         "bytes_per_launch": 2e9, "flops_per_launch": 0.0},
        {"name": "near+project", "kernel": "k_gemm_lds<0, 8, 2, 0>", "total_ms": 4.0, "launches": 1,
         "bytes_per_launch": 1e9, "flops_per_launch": 314e9},
    ]
    g = bench.kernel_table(stages, (2, 2), 16, True)
    agg = g["k_agg_stream<float, 6, 32>"]
    assert agg["launches"] == 2 and agg["bound"] == "hbm" and agg["bytes"] == pytest.approx(6e9)
    assert g["k_gemm_lds<0, 8, 2, 0>"]["bound"] == "mfma"
    r = bench.kernel_roofline(agg)               # 6 GB in 3 ms = 2 TB/s
    assert r["achieved"] == pytest.approx(2000.0) and r["frac"] == pytest.approx(0.25)
    m = bench.kernel_roofline(g["k_gemm_lds<0, 8, 2, 0>"])
    assert m["unit"] == "TFLOP/s" and m["achieved"] == pytest.approx(78.5)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_traffic_follows_the_kernel_source(tmp_path, monkeypatch):
    """bench.py reports counter traffic for a kernel only from a digest
    taken on the same engine source: the bytes per launch while the hash
    matches, None once the source has changed or the digest is missing."""
    rec = {"workload": "c5", "source_sha256": "abc", "calibration": {"fetch_scale": 2.0, "write_scale": 1.0},
           "kernels": {"k_translate_reg<2, false>": {"dispatches": 12, "fetch_bytes_per_launch": 3.0e9,
                                                    "write_bytes_per_launch": 1.0e9,
                                                    "traffic_bytes_per_launch": 4.0e9}}}
    path = tmp_path / "pmc_traffic_c5_r16.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "traffic_file", lambda workload, R: str(path))
    monkeypatch.setattr(bench, "source_digest", lambda: "abc")
    assert bench.measured_traffic("k_translate_reg<2, false>", "c5", 16) == pytest.approx(4.0e9)
    assert bench.measured_traffic("k_agg_stream<float, 6, 32, 2>", "c5", 16) is None
    monkeypatch.setattr(bench, "source_digest", lambda: "def")
    assert bench.measured_traffic("k_translate_reg<2, false>", "c5", 16) is None
    monkeypatch.setattr(bench, "traffic_file", lambda workload, R: str(tmp_path / "missing.json"))
    monkeypatch.setattr(bench, "source_digest", lambda: "abc")
    assert bench.measured_traffic("k_translate_reg<2, false>", "c5", 16) is None
