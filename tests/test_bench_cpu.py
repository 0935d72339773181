"""bench.py contract checks that need no GPU."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU only" in msg["error"]


def test_lane_op_model_counts_every_unit():
    sys.path.insert(0, ROOT)
    import bench
    u = {"filter_words": 7, "triple_tests": 10, "gen_nodes": 100, "verify_tests": 1000}
    # per node at t = 3: 4 * (3 pairs + 1 triple); at t = 4: 4 * (6 + 4)
    assert bench.lane_ops(u, 3) == 2 * 7 + 14 * 10 + 16 * 100 + 5 * 1000
    assert bench.lane_ops(u, 4) == 2 * 7 + 14 * 10 + 40 * 100 + 5 * 1000
