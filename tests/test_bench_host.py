"""Host logic of the benchmark line (no GPU): the measured HBM traffic enters
the line only while the kernel source is the one the counters were taken on,
scaled to the launch's work units, and more than one GPU is refused."""
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_committed_traffic_scales_with_the_launch():
    src = os.path.join(ROOT, "paper_2108_10480_amd", "csrc", "eval.hip")
    t = json.load(open(os.path.join(ROOT, "profiles", "traffic_k_eval_icosphere_l7_1M.json")))
    if t["source_sha"] != bench._sha(src):
        assert bench._traffic(src, "traffic_k_eval_icosphere_l7_1M.json", 1000000) is None
        pytest.skip("the kernel source changed since its counters were taken (the line reports null)")
    b = bench._traffic(src, "traffic_k_eval_icosphere_l7_1M.json", t["units_per_launch"])
    assert b == t["hbm_bytes_per_launch"]
    assert bench._traffic(src, "traffic_k_eval_icosphere_l7_1M.json", 2 * t["units_per_launch"]) == 2 * b
    # FETCH and WRITE in KiB per dispatch, each with its copy-kernel scale
    assert abs(1024 * (t["fetch_kib_per_dispatch"] * t["fetch_scale"] + t["write_kib_per_dispatch"] *
                       t["write_scale"]) - t["hbm_bytes_per_launch"]) <= 1e-6 * t["hbm_bytes_per_launch"]


def test_traffic_is_null_for_a_changed_source(tmp_path):
    changed = tmp_path / "eval.hip"
    changed.write_bytes(open(os.path.join(ROOT, "paper_2108_10480_amd", "csrc", "eval.hip"), "rb").read() + b"\n")
    assert bench._traffic(str(changed), "traffic_k_eval_icosphere_l7_1M.json", 1000000) is None
    assert bench._traffic(str(changed), "no_such_summary.json", 1000000) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr and r.stdout == ""
