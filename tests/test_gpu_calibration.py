"""The mixed solve's stopping tolerance (FP64 residual 2e-9, the benchmark
default) gives a relative L2 error below 1e-6 against the FP64 oracle: the
512^3 workload's recipe (BBKS prior, 500 Mpc box, cap mask, lognormal-Poisson
galaxies, TSC with 2x supersampling) at 128^3."""
import os
import sys

import numpy as np
import pytest

import synth
from oracle import wiener as ow

from gpu_util import context, rel_l2

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_error_at_benchmark_tolerance():
    import bench
    wl = synth.workload("bbks512", n=128)
    ptab = wl.ptab()
    w = wl.mask()
    cat = wl.catalogue(ptab, w)
    res = ow.reconstruct(cat.xyz, wl.n, wl.box, w, ptab, wl.scheme, wl.supersample, 1e-11, 20000,
                         workers=8)
    assert res["status"] == "ok"
    ctx = context()
    ctx.set_grid(wl.n, wl.box)
    ctx.set_mask(w)
    ctx.set_power(ptab)
    ctx.set_galaxies(cat.xyz)
    ctx.deposit(wl.scheme, wl.supersample)
    x, info = ctx.solve(precision="mixed", tol=bench.DEFAULT_TOL, max_iter=100000)
    err = rel_l2(x, res["x"])
    print(f"calibration 128^3: rel_res_true={info.rel_res_true:.3e} err={err:.3e} "
          f"ratio={err / info.rel_res_true:.1f} iters={info.iters_total}")
    assert info.rel_res_true <= bench.DEFAULT_TOL
    assert err < 1e-6
    ctx.close()
