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


@pytest.mark.parametrize("n,nrhs", [(64, 4), (128, 2)])
def test_batch_rhs_against_oracle(n, nrhs):
    """The batch workload's recipe (BBKS prior, 500 Mpc box, cap mask, CIC on
    the 2x grid, mixed prior-split CG to the benchmark's split residual
    3e-7): every RHS of the batch within 1e-6 relative L2 of the oracle's
    A^-1 b (its split CG to 1e-12)."""
    wl = synth.workload("bbks256", n=n)
    ptab = wl.ptab()
    w = wl.mask()
    cats = []
    for j in range(nrhs):
        wl.seed = 4000 + 3 * j
        cats.append(wl.catalogue(ptab, w).xyz)
    ctx = context()
    ctx.set_grid(n, wl.box)
    ctx.set_mask(w)
    ctx.set_power(ptab)
    outs, infos = ctx.solve_batch(cats, "cic", 2, precision="mixed", precond="prior", tol=3e-7,
                                  max_iter=100000)
    ctx.close()
    for j, (xyz, x, info) in enumerate(zip(cats, outs, infos)):
        assert info.status == 0
        res = ow.reconstruct(xyz, n, wl.box, w, ptab, "cic", 2, 0.0, 0, workers=16)
        ref = ow.split_cg(res["system"], res["b"], 1e-12, 100000)
        err = rel_l2(x, ref["x"])
        print(f"batch {n}^3 rhs {j}: {len(xyz)} galaxies, {info.iters_total} iterations, "
              f"error {err:.3e}")
        assert err < 1e-6
