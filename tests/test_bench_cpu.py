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


def test_sample_errors_keep_the_worst_error_per_row_field():
    import numpy as np
    sys.path.insert(0, ROOT)
    import bench
    import oracle
    rng = np.random.default_rng(0)
    H = ((rng.standard_normal((4, 16)) + 1j * rng.standard_normal((4, 16))) / np.sqrt(2)).astype(np.complex64)
    xi = 0.5
    X, Wd, _ = oracle.direct_rzf(H.T.astype(np.complex128), xi)
    WT = oracle.rzf(H.T.astype(np.complex128), xi, tol=0.0, max_iter=2)["W"]
    rows = {"a": {"b": {}}}
    samples = [dict(path=("a", "b"), H=H, xi=xi, T=2, checks=[("w", "W_fp64", Wd), ("x", "X_fp64", X * 1.01),
                                                             ("t", "W_oracle_T", WT)]),
               dict(path=("a", "b"), H=H, xi=xi, T=2, checks=[("w", "W_fp64", Wd * (1 + 1e-3))])]
    bench.sample_errors(samples, rows)
    r = rows["a"]["b"]
    assert abs(r["w"] - 1e-3) < 1e-9 and abs(r["x"] - 1e-2) < 1e-9 and r["t"] == 0.0


def test_busy_summary_from_counters(tmp_path):
    sys.path.insert(0, ROOT)
    from paper_2305_13925_amd import profile_summary as ps
    d = tmp_path / "pmc"
    d.mkdir()
    head = ('"Dispatch_Id","Grid_Size","Kernel_Name","Counter_Name","Counter_Value","Start_Timestamp",'
            '"End_Timestamp"\n')
    name = "void jacpcg::(anonymous namespace)::gram_bf16_small_kernel<3, 2, true>(jacpcg::GramLaunch)"
    # 100 us dispatch, 2e5 cycles per XCD (2 GHz), MFMA busy on half of the SIMD cycles
    body = (f'1,262144,"{name}","GRBM_GUI_ACTIVE",{8 * 2e5},1000000,1100000\n'
            f'1,262144,"{name}","SQ_VALU_MFMA_BUSY_CYCLES",{1024 * 1e5},1000000,1100000\n')
    (d / "p_counter_collection.csv").write_text(head + body)
    (d / "p_agent_info.csv").write_text('"Simd_Count","Num_Xcc"\n0,0\n1024,8\n')
    out = tmp_path / "busy"
    ps.main(["busy", str(d), "--cmd", "x", "--out", str(out)])
    import json
    rec = json.load(open(str(out) + ".json"))
    assert abs(rec["gram"]["clock_ghz"] - 2.0) < 1e-9 and abs(rec["gram"]["mfma_busy"] - 0.5) < 1e-9
