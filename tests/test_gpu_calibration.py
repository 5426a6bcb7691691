"""The mixed solve's stopping tolerances (the benchmark's, per
preconditioning) give a relative L2 error below 1e-6 against the FP64 oracle:
the 512^3 workload's recipe (BBKS prior, 500 Mpc box, cap mask,
lognormal-Poisson galaxies, TSC with 2x supersampling) at 128^3."""
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


@pytest.fixture(scope="module")
def case128():
    wl = synth.workload("bbks512", n=128)
    ptab = wl.ptab()
    w = wl.mask()
    cat = wl.catalogue(ptab, w)
    res = ow.reconstruct(cat.xyz, wl.n, wl.box, w, ptab, wl.scheme, wl.supersample, 1e-11, 20000,
                         workers=8)
    assert res["status"] == "ok"
    return wl, ptab, w, cat, res


@pytest.mark.parametrize("precond", ["none", "prior"])
def test_error_at_benchmark_tolerance(case128, precond):
    import bench
    wl, ptab, w, cat, res = case128
    tol = bench.TOLERANCES[precond]
    ctx = context()
    ctx.set_grid(wl.n, wl.box)
    ctx.set_mask(w)
    ctx.set_power(ptab)
    ctx.set_galaxies(cat.xyz)
    ctx.deposit(wl.scheme, wl.supersample)
    x, info = ctx.solve(precision="mixed", tol=tol, max_iter=100000, precond=precond)
    err = rel_l2(x, res["x"])
    sysm, b = res["system"], res["b"]
    if precond == "prior":
        # the split residual the solve stopped on, recomputed by the oracle
        sp = ow.SplitSystem(sysm)
        stop = float(np.linalg.norm(sp.split(b - sysm.apply(x))) / np.linalg.norm(sp.split(b)))
    else:
        stop = float(np.linalg.norm(b - sysm.apply(x)) / np.linalg.norm(b))
    print(f"calibration 128^3 {precond}: stop residual {stop:.3e} "
          f"rel_res_true={info.rel_res_true:.3e} err={err:.3e} iters={info.iters_total}")
    assert stop <= 1.01 * tol
    assert err < 1e-6
    ctx.close()
