"""Host-side checks of bench.py that need no GPU."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus_requested"] == 2 and "one GPU" in msg["error"]


def test_profiled_traffic_is_reported_only_for_the_profiled_kernel_and_workload():
    for name in bench.PROFILED_TRAFFIC:
        assert bench.profiled_traffic(name, default_workload=False) is None
        got = bench.profiled_traffic(name, default_workload=True)
        # the table is keyed by the kernel source hash: a stale entry reads None
        assert got is None or got == bench.PROFILED_TRAFFIC[name]["bytes"]
        assert os.path.exists(os.path.join(ROOT, bench.PROFILED_TRAFFIC[name]["profile"]))
    assert bench.profiled_traffic("no_such_kernel", default_workload=True) is None
