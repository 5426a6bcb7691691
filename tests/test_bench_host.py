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


def test_cpu_baseline_phases_on_a_small_workload():
    """The oracle's per-phase timing on a 16^3 version of the headline recipe:
    every phase is timed, the CG iteration is extrapolated and labelled."""
    import synth
    wl = synth.workload("bbks512", n=16)
    wl.n_target = 5000
    ptab = wl.ptab()
    w = wl.mask()
    xyz = wl.catalogue(ptab, w).xyz
    for precond in ("prior", "none"):
        base = bench.cpu_baseline(wl, ptab, w, xyz, 40, precond, cg_iters=4)
        ph = base["phases_s"]
        assert base["kind"] == "oracle" and base["extrapolated"]
        assert base["cores"] >= 1 and base["value"] > 0
        assert ph["cg_iterations_timed"] == 4 and ph["cg_iterations_extrapolated"] == 40
        assert min(ph["deposit"], ph["lowpass"], ph["cg_iteration"]) > 0
        total = ph["deposit"] + ph["lowpass"] + ph["data_vector"] + 40 * ph["cg_iteration"]
        # the phases are reported rounded (1 ms, the iteration 0.1 ms)
        assert abs(1.0 / base["value"] - total) < 0.01 * total + 3 * 5e-4 + 40 * 5e-5
