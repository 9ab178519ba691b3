"""bench.py's host-side contract (no GPU needed)."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_algorithmic_work_of_the_headline_shape():
    sys.path.insert(0, ROOT)
    import bench
    a = bench.algorithmic(1024, 64, 64, 8, 1024, "bf16x6", "split")
    # Gram: 4 M K (K + 1) flops and 8 M K + 8 K^2 bytes per instance
    assert a["gram"]["flops"] == 1024 * 4.0 * 1024 * 64 * 65
    assert a["gram"]["bytes"] == 1024 * (8.0 * 1024 * 64 + 8.0 * 64 * 64)
    # precoder: 8 M K n flops, H and X read, W written
    assert a["epilogue"]["bytes"] == 1024 * (8.0 * 1024 * 64 * 2 + 8.0 * 64 * 64)
    bound, t = bench.binding_roof(a["epilogue"])
    assert bound == "hbm" and abs(t - a["epilogue"]["bytes"] / 8e12) < 1e-12
