"""Multi-RHS batch: one launch per pass covers every right-hand side; each
result equals the single-RHS solve of the same catalogue bit for bit, and the
oracle to the solve tolerance."""
import numpy as np
import pytest

import synth
from oracle import wiener as ow

from gpu_util import context, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def batch():
    wl = synth.Workload("b32", 32, 300.0, "cic", 2, 30000, 401, "bbks")
    ptab = wl.ptab()
    w = wl.mask()
    cats = []
    for j in range(4):
        wl.seed = 401 + 3 * j
        cats.append(wl.catalogue(ptab, w).xyz)
    cats.append(np.zeros((0, 3)))  # an empty catalogue: zero right-hand side
    return wl, ptab, w, cats


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_batch_equals_single(batch, prec):
    wl, ptab, w, cats = batch
    ctx = context()
    ctx.set_grid(wl.n, wl.box)
    ctx.set_mask(w)
    ctx.set_power(ptab)
    outs, infos = ctx.solve_batch(cats, "cic", 2, precision=prec, tol=1e-10, max_iter=20000)
    for xyz, x, info in zip(cats, outs, infos):
        assert info.status == 0
        ctx.set_galaxies(xyz)
        ctx.deposit("cic", 2)
        y, inf1 = ctx.solve(precision=prec, tol=1e-10, max_iter=20000)
        assert np.array_equal(x, y)
        assert info.iters_total == inf1.iters_total
    assert not outs[-1].any()
    res = ow.reconstruct(cats[1], wl.n, wl.box, w, ptab, "cic", 2, 1e-12, 20000)
    assert rel_l2(outs[1], res["x"]) < 1e-6
    ctx.close()
