"""bench.py's contract checks that need no GPU."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_roofline_work_formulas():
    sys.path.insert(0, ROOT)
    import bench
    amt, unit, bound, peak = bench.step_work("update_W", 26000, 11000, 200, 857250)
    assert unit == "flop" and bound == "mfma" and amt == 2.0 * 26000 * 200 * 200
    amt, unit, bound, peak = bench.step_work("product_R", 26000, 11000, 200, 857250)
    assert unit == "byte" and bound == "hbm"
    assert amt == 8.0 * 857250 + 4.0 * 11001 + 4.0 * 200 * (11000 + 26000)


def test_counters_file_is_valid_json_if_present():
    p = os.path.join(ROOT, "profiles", "counters.json")
    if os.path.exists(p):
        c = json.load(open(p))
        assert "source_digest" in c and "entries" in c
