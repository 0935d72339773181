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


def test_traffic_record_is_consistent():
    # HBM bytes per launch = FETCH_SIZE and WRITE_SIZE (KiB per dispatch pair)
    # scaled by what the same counters read for a copy of known size
    sys.path.insert(0, ROOT)
    import bench
    with open(bench.TRAFFIC_FILE) as f:
        t = json.load(f)
    cal = t["copy_calibration"]
    assert abs(cal["fetch_factor"] - cal["bytes"] / (cal["fetch_size_kib"] * 1024)) < 1e-9
    assert abs(cal["write_factor"] - cal["bytes"] / (cal["write_size_kib"] * 1024)) < 1e-9
    assert abs(t["fetch_bytes"] - t["fetch_size_kib"] * 1024 * cal["fetch_factor"]) < 1e3
    assert abs(t["write_bytes"] - t["write_size_kib"] * 1024 * cal["write_factor"]) < 1e3
    assert t["hbm_bytes_per_launch"] == t["fetch_bytes"] + t["write_bytes"]
    # the record only counts while the kernel and launch sources are the ones measured
    assert (bench.load_traffic() is not None) == (t["kernel_source_sha256"] == bench.kernel_sha256())
