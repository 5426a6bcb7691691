"""bench.py end to end on a small grid: one JSON line with the fields of its
contract (roofline and CPU baseline objects included)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.gpu
def test_bench_json_contract():
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--n", "64", "--steps", "2",
           "--warmup", "1", "--serve", "0", "--batch", "0", "--sd", "0", "--no-post",
           "--configs", "0", "--deposit-stress", "0"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=200, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    d = json.loads(r.stdout.strip().splitlines()[-1])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
              "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1
    assert d["value"] > 0 and d["unit"] == "solves/s" and d["higher_is_better"] is True
    assert "workload" in d["config"] and d["config"]["n"] == 64
    rf = d["roofline"]
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert 0 < rf["frac"] < 1 and abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-3
    assert "traffic" in rf
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] >= 1 and cb["value"] > 0
    assert cb["unit"] == "solves/s" and cb["sample"] and cb["extrapolated"]
    assert set(cb["phases_s"]) >= {"deposit", "lowpass", "data_vector", "cg_iteration"}
