"""Host-side pieces of bench.py (no GPU): the one-GPU guard, the profile
traffic lookup keyed by the kernel sources, and the host description."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_traffic_follows_the_kernel_sources():
    path = os.path.join(ROOT, "profiles", "traffic.json")
    with open(path) as fh:
        t = json.load(fh)
    k, ent = next(iter(t.items()))
    if ent["kernel_hash"] == bench.kernel_hash():
        assert bench.traffic_for(k, 1.0) == ent["bytes_per_launch"]
    assert bench.traffic_for("no such kernel", 1.0) is None


def test_host_cpu():
    h = bench.host_cpu()
    assert h["nproc"] >= 1
