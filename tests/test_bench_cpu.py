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
    """The per-site VALU count adds up from its parts (see the docstring)."""
    sys.path.insert(0, ROOT)
    import bench
    thermal = 40 + 8 + 6 + 3 + 3
    stage = lambda exch: exch + 4 + 18
    ops = thermal + 3 + stage(18) * 2 + 10 + 13
    assert ops == 166
    assert bench.alu_cycles_per_site("fp32", "slab") == ops - 9 + 9 * 4
    assert bench.alu_cycles_per_site("fp32", "l10") == ops + 2 * (54 - 18) - 9 + 9 * 4
    assert bench.alu_cycles_per_site("fp64", "slab") is None
    assert abs(bench.VALU_PEAK_T - 39.3216) < 1e-9
