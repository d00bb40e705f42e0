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


def test_profiled_traffic_is_reported_only_for_the_profiled_kernel_ac_and_workload():
    for name, ent in bench.PROFILED_TRAFFIC.items():
        blob = b"an AC that was not profiled"
        assert bench.profiled_traffic(name, False, blob) is None
        assert bench.profiled_traffic(name, True, blob) is None
        # keyed by the kernel source hash and the AC's hash: a stale entry reads None
        assert bench.kernel_sha16() != ent["kernel_sha256_16"] or ent["bytes"] > 0
        assert os.path.exists(os.path.join(ROOT, ent["profile"]))
        with open(os.path.join(ROOT, ent["profile"])) as f:
            text = f.read()
        assert ent["kernel_sha256_16"] in text and ent["ac_sha256_16"] in text
    assert bench.profiled_traffic("no_such_kernel", True, b"") is None
