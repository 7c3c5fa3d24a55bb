"""bench.py contract checks that need no GPU."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_alu_work_count():
    """The per-site VALU count adds up from its parts (see the docstring), and
    the peak is the published FP32 vector rate in FMAs."""
    sys.path.insert(0, ROOT)
    import bench
    thermal = 40 + 8 + 6 + 3 + 3
    stage = lambda exch: exch + 4 + 18
    ops = thermal + 3 + stage(18) * 2 + 10 + 13
    assert ops == 166
    weigh = lambda n: n - 20 - 9 + 20 * bench.W_PRODUCT + 9 * bench.W_TRANS
    assert abs(bench.alu_ops_per_site("fp32", "slab") - weigh(ops)) < 1e-9
    assert abs(bench.alu_ops_per_site("fp32", "l10") - weigh(ops + 2 * (54 - 18))) < 1e-9
    assert bench.alu_ops_per_site("fp64", "slab") is None
    assert abs(bench.VALU_PEAK_T - 157.2864 / 2) < 1e-9
    mc = 40 + 6 + (2 + 1) + (2 + 2) + 18 + 3 + 11 + (3 + 1)
    assert mc == 89 and abs(bench.MC_ALU_OPS - (mc - 20 - 4 + 20 * bench.W_PRODUCT
                                                 + 4 * bench.W_TRANS)) < 1e-9


def test_issue_rate_calibration_library_loads(tmp_path):
    """The benchmark's VALU issue-rate calibration is a measurement probe built on
    demand into its own library (never part of the step library); it loads and
    names its classes without a GPU."""
    import ctypes
    sys.path.insert(0, ROOT)
    from paper_2502_02236_amd import build as B
    src = os.path.join(ROOT, "tests", "helpers", "issue_rate.hip")
    lib = ctypes.CDLL(B.build_probe(src, str(tmp_path / "libissue_rate.so")))
    lib.issue_rate_name.restype = ctypes.c_char_p
    names = [lib.issue_rate_name(k).decode() for k in range(lib.issue_rate_classes())]
    assert names[0] == "v_fma_f32" and "v_mad_u64_u32" in names and "v_log_f32" in names
    assert lib.issue_rate_name(len(names)) is None and lib.issue_rate_chains() == 8
    f = ctypes.c_float()
    assert lib.issue_rate_time(-1, None, 1, 1, ctypes.byref(f)) == -1
    from paper_2502_02236_amd import asd as A
    assert not hasattr(A.lib(), "issue_rate_time")
    assert not any("issue_rate" in src for src, _ in B.SOURCES)


def test_graph_segments_time_exactly_the_requested_steps():
    sys.path.insert(0, ROOT)
    import bench
    assert bench.segment_steps(2000) == 1000
    assert bench.segment_steps(20) == 20
    assert bench.segment_steps(300) == 300
    assert bench.segment_steps(2100) == 700
    assert bench.segment_steps(25) == 24      # odd: 24 in a graph, one eager step
    assert bench.segment_steps(1) == 0
    for k in (2, 7, 64, 999, 1000, 3000, 4097):
        g = bench.segment_steps(k)
        assert g % 2 == 0 and g <= 1000 and (g == 0 or k - (k // g) * g <= 1)


def test_cpu_baseline_worker_runs_the_cropped_track():
    """One oracle worker on the cropped track window (a few steps): it counts
    the magnetic window sites of the crop and times only the steps."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--cpu-worker", "1",
                        "--cpu-steps", "2"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["updates"] == 2 * out["magnetic_sites"]
    assert 0.5 * 64 * 64 * 33 < out["magnetic_sites"] < 64 * 64 * 33
    assert out["seconds"] > 0
