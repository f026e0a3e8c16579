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


def _traffic_files():
    d = os.path.join(ROOT, "profiles")
    return sorted(f for f in os.listdir(d) if f.startswith("traffic_") and f.endswith(".json"))


@pytest.mark.parametrize("name", _traffic_files())
def test_committed_traffic_scales_with_the_launch(name):
    t = json.load(open(os.path.join(ROOT, "profiles", name)))
    src = os.path.join(ROOT, "paper_2108_10480_amd", "csrc", t["source_file"])
    if t["source_sha"] != bench._sha(src):
        assert bench._traffic(src, name, 1000000) is None
        pytest.skip("the kernel source changed since its counters were taken (the line reports null)")
    b = bench._traffic(src, name, t["units_per_launch"])
    assert b == t["hbm_bytes_per_launch"]
    assert bench._traffic(src, name, 2 * t["units_per_launch"]) == 2 * b
    # FETCH and WRITE in KiB per dispatch, each with its copy-kernel scale
    assert abs(1024 * (t["fetch_kib_per_dispatch"] * t["fetch_scale"] + t["write_kib_per_dispatch"] *
                       t["write_scale"]) - t["hbm_bytes_per_launch"]) <= 1e-6 * t["hbm_bytes_per_launch"]


def test_work_model_counts_every_term_once():
    """FLOPs and bytes per query: 20 and 32 per node, 25 per far-field term,
    30 / 80 / 200 FLOPs and 12 / 32 / 40 bytes per point / edge / triangle
    leaf, plus 28 bytes of query and results."""
    import numpy as np
    cnt = np.array([[100, 40, 3, 2, 1], [300, 60, 5, 0, 7]], np.int64)
    work, flops, nbytes = bench._work(np, cnt)
    assert work["nodes"] == 200 and work["far_terms"] == 50
    assert flops == 20 * 200 + 25 * 50 + 30 * 4 + 80 * 1 + 200 * 4
    assert nbytes == 28 + 32 * 200 + 12 * 4 + 32 * 1 + 40 * 4
    r = bench._roofline("k", 1000, 2.0, flops, nbytes, traffic=8e6)
    assert abs(r["achieved"] - 1000 * flops / 2e-3 / 1e12) < 1e-12
    assert r["frac"] == r["achieved"] / bench.ALU_PEAK_TFLOPS
    assert abs(r["hbm_measured"]["achieved"] - 8e6 / 2e-3 / 1e9) < 1e-9
    assert "frac" not in r["algorithmic_bytes"]


def test_traffic_is_null_for_a_changed_source(tmp_path):
    changed = tmp_path / "eval.hip"
    changed.write_bytes(open(os.path.join(ROOT, "paper_2108_10480_amd", "csrc", "eval.hip"), "rb").read() + b"\n")
    for name in _traffic_files():
        assert bench._traffic(str(changed), name, 1000000) is None
    assert bench._traffic(str(changed), "no_such_summary.json", 1000000) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr and r.stdout == ""
