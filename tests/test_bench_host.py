"""Host-side pieces of bench.py: the algorithmic-bytes formulas (Algorithm
1's step, the kept-walk output), the counter-traffic lookup, the host CPU
description, and the one-GPU contract."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_algorithmic_bytes_by_hand():
    # 10 draws, 3 of them finding no live edge; 4 ids in 2 kept walks:
    # 17 B per draw, 12 more per live edge, 4 per id, 20 per kept walk
    st = {"steps": 10, "dead_ends": 3, "walk_ids": 4, "hits": 2}
    assert bench.algorithmic_bytes(st) == 17 * 10 + 12 * 7 + 4 * 4 + 20 * 2
    # the flat reading: a fixed price per step, 4 B per attempt, 4 per id, 16 per walk
    assert bench.per_step_bytes(st, 100, 29) == 29 * 10 + 4 * 100 + 4 * 4 + 16 * 2
    assert bench.per_step_bytes(st, 100, 21) == 21 * 10 + 4 * 100 + 4 * 4 + 16 * 2


def test_traffic_only_for_its_query_and_kernel():
    with open(bench.TRAFFIC_FILE) as f:
        t = json.load(f)
    q = (t["workload"], t["mode"], t["n_attempts"], t["cycle_steps"])
    got = bench.load_traffic(*q)
    if t["kernel_sha"] == bench.kernel_sha():
        assert got == t
        assert t["traffic_bytes_per_launch"] == t["fetch_bytes_per_launch"] + t["write_bytes_per_launch"]
    else:
        assert got == {}
    other_mode = "nodes" if t["mode"] == "edges" else "edges"
    assert bench.load_traffic("another workload", *q[1:]) == {}
    assert bench.load_traffic(q[0], other_mode, *q[2:]) == {}
    assert bench.load_traffic(q[0], q[1], q[2] // 2, q[3]) == {}
    assert bench.load_traffic(*q[:3], not q[3]) == {}


def test_host_cpu_fields():
    model, logical, physical = bench.host_cpu()
    assert isinstance(model, str) and logical >= 1 and physical >= 1


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""
