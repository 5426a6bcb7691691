"""GPU parity of the CG solves against the oracle (through the C ABI)."""
import numpy as np
import pytest

import synth
from oracle import wiener as ow

from gpu_util import context, rel_l2
import sensitivity as se

pytestmark = pytest.mark.gpu

WF_OK, WF_EINVAL, WF_ESTATE, WF_ENOTCONV, WF_EOVERFLOW = 0, 1, 2, 5, 6


@pytest.fixture(scope="module")
def ctx():
    c = context()
    yield c
    c.close()


@pytest.fixture(scope="module")
def pl32():
    """32^3 / 256 Mpc power-law workload, NGP, oracle reference solution."""
    wl = synth.workload("pl32")
    ptab = wl.ptab()
    w = wl.mask()
    cat = wl.catalogue(ptab, w)
    res = ow.reconstruct(cat.xyz, wl.n, wl.box, w, ptab, "ngp", 1, 1e-10, 5000)
    ref = ow.reference_solution(res["system"], res["b"], tol=1e-14)
    return dict(wl=wl, ptab=ptab, w=w, xyz=cat.xyz, res=res, x_ref=ref["x"])


def _load(ctx, d):
    wl = d["wl"]
    ctx.set_grid(wl.n, wl.box)
    ctx.set_mask(d["w"])
    ctx.set_power(d["ptab"])
    ctx.set_galaxies(d["xyz"])
    ctx.deposit("ngp", 1)


def test_data_vector_matches_oracle(ctx, pl32):
    _load(ctx, pl32)
    _, nobs, nbar = ctx.get_deposit(False, True, 1)
    assert nbar == pytest.approx(pl32["res"]["nbar"], rel=1e-15)
    assert np.array_equal(nobs, pl32["res"]["n_obs"])


@pytest.fixture(scope="module")
def bbks48():
    """48^3 / 500 Mpc, BBKS prior, 60 deg cap with exp(-r/150 Mpc), lognormal
    Poisson catalogue with 2x supersampled CIC: a problem whose fixed-k CG
    iterates are stable under rounding (the oracle's own iterate moves by
    7e-10 at k = 50 and 3e-13 at k = 300 under rounding-sized noise,
    tests/sensitivity.py)."""
    wl = synth.Workload("bbks48", 48, 500.0, "cic", 2, 60000, 211, "bbks")
    ptab = wl.ptab()
    w = wl.mask()
    cat = wl.catalogue(ptab, w)
    res = ow.reconstruct(cat.xyz, wl.n, wl.box, w, ptab, "cic", 2, 1e-10, 5000)
    return dict(wl=wl, ptab=ptab, w=w, xyz=cat.xyz, res=res)


@pytest.mark.parametrize("k", [50, 300])
def test_fixed_iteration_parity_fp64(ctx, bbks48, k):
    """Both sides run exactly k CG iterations from x = 0; the bound is a
    multiple of the oracle's own spread at that k under rounding-sized noise
    (tests/sensitivity.py)."""
    tol = se.bound("bbks48", "plain", k)
    d = bbks48
    wl = d["wl"]
    ctx.set_grid(wl.n, wl.box)
    ctx.set_mask(d["w"])
    ctx.set_power(d["ptab"])
    ctx.set_galaxies(d["xyz"])
    ctx.deposit("cic", 2)
    x, info = ctx.solve(precision="fp64", tol=0.0, max_iter=k, allow=(WF_ENOTCONV,))
    assert info.iters_total == k and info.status == WF_ENOTCONV
    ref = ow.cg(d["res"]["system"], d["res"]["b"], 0.0, k)
    err = rel_l2(x, ref["x"])
    print(f"bbks48 plain k={k}: rel L2 {err:.3e}, bound {tol:.1e} "
          f"({err / se.SPREADS[('bbks48', 'plain', k)]:.2f} x the oracle's spread)")
    assert err < tol
    assert info.rel_res_recursive == pytest.approx(ref["rel_res"], rel=max(tol, 1e-9))


@pytest.mark.parametrize("k", [50, 300])
def test_fixed_iteration_parity_powerlaw(ctx, pl32, k):
    """The power law with its Gaussian cut-off isolates the largest
    eigenvalues (the corner modes); fixed-k CG iterates are rounding-chaotic
    there: the oracle's own k-th iterate moves by 3e-5 (k = 50) and 2e-6
    (k = 300) under rounding-sized noise (tests/sensitivity.py), and the
    bound is a multiple of that; the converged comparison below is the tight
    one."""
    tol = se.bound("pl32", "plain", k)
    _load(ctx, pl32)
    x, info = ctx.solve(precision="fp64", tol=0.0, max_iter=k, allow=(WF_ENOTCONV,))
    assert info.iters_total == k
    ref = ow.cg(pl32["res"]["system"], pl32["res"]["b"], 0.0, k)
    err = rel_l2(x, ref["x"])
    print(f"pl32 plain k={k}: rel L2 {err:.3e}, bound {tol:.1e} "
          f"({err / se.SPREADS[('pl32', 'plain', k)]:.2f} x the oracle's spread)")
    assert err < tol


def test_converged_solve_fp64(ctx, pl32):
    _load(ctx, pl32)
    x, info = ctx.solve(precision="fp64", tol=1e-10, max_iter=5000)
    r = pl32["res"]
    assert info.status == WF_OK
    assert abs(info.iters_total - r["iterations"]) <= 3
    assert info.rel_res_true < 2e-10
    e_gpu = rel_l2(x, pl32["x_ref"])
    e_or = rel_l2(r["x"], pl32["x_ref"])
    assert e_gpu <= 2 * e_or + 1e-12


def test_mixed_solve_error(ctx, pl32):
    _load(ctx, pl32)
    x, info = ctx.solve(precision="mixed", tol=1e-10, max_iter=20000)
    assert info.status == WF_OK
    assert info.outer_steps >= 2
    assert info.rel_res_true <= 1e-10
    assert rel_l2(x, pl32["x_ref"]) < 1e-6


def test_zero_rhs_gives_zero(ctx):
    n = 16
    ctx.set_grid(n, 100.0)
    ctx.set_mask(np.full((n, n, n), 0.7))
    ctx.set_power(synth.p_by_m2(lambda k: synth.bbks_power(k), n, 100.0))
    ctx.set_rhs(np.zeros((n, n, n)), 1.0)
    for prec in ("fp64", "mixed"):
        x, info = ctx.solve(precision=prec, tol=1e-8, max_iter=100)
        assert info.status == WF_OK and not x.any()


def test_invalid_inputs_are_rejected(ctx):
    import paper_0906_3978_amd as wf
    with pytest.raises(wf.WienerError) as e:
        ctx.set_grid(20, 100.0)
    assert e.value.code == WF_EINVAL
    n = 16
    ctx.set_grid(n, 100.0)
    bad = np.full((n, n, n), 0.5)
    bad[1, 2, 3] = 1.5
    with pytest.raises(wf.WienerError) as e:
        ctx.set_mask(bad)
    assert e.value.code == WF_EINVAL
    with pytest.raises(wf.WienerError) as e:
        ctx.set_mask(np.zeros((n, n, n)))
    assert e.value.code == WF_EINVAL
    p = synth.p_by_m2(lambda k: synth.bbks_power(k), n, 100.0)
    p[7] = -1.0
    with pytest.raises(wf.WienerError) as e:
        ctx.set_power(p)
    assert e.value.code == WF_EINVAL
    with pytest.raises(wf.WienerError) as e:
        ctx.set_power(p[:-1])
    assert e.value.code == WF_EINVAL
    with pytest.raises(wf.WienerError) as e:
        ctx.set_galaxies(np.array([[1.0, 2.0, 100.0]]))
    assert e.value.code == WF_EINVAL
    with pytest.raises(wf.WienerError) as e:
        ctx.set_galaxies(np.array([[1.0, np.nan, 3.0]]))
    assert e.value.code == WF_EINVAL
    with pytest.raises(wf.WienerError) as e:
        ctx.solve(precision="fp64", tol=1e-6, max_iter=10)
    assert e.value.code == WF_ESTATE


def test_too_many_galaxies_overflow(ctx):
    import ctypes
    import paper_0906_3978_amd as wf
    ctx.set_grid(16, 100.0)
    L = wf.lib()
    dummy = np.zeros(3)
    code = L.wf_set_galaxies(ctx._h, dummy.ctypes.data, 1 << 24, 0)
    assert code == WF_EOVERFLOW


def test_not_converged_returns_last_iterate(ctx, pl32):
    _load(ctx, pl32)
    x, info = ctx.solve(precision="fp64", tol=1e-12, max_iter=1, allow=(WF_ENOTCONV,))
    assert info.status == WF_ENOTCONV and info.iters_total == 1
    ref = ow.cg(pl32["res"]["system"], pl32["res"]["b"], 0.0, 1)
    assert rel_l2(x, ref["x"]) < 1e-13


def test_snapshot_resume_bit_identical(ctx, pl32):
    _load(ctx, pl32)
    ctx.solve_begin(precision="fp64", tol=1e-10, max_iter=5000)
    ctx.solve_step(40)
    snap = ctx.snapshot()
    ctx.solve_step(60)
    x_direct, _ = ctx.solve_finish(allow=(WF_OK, WF_ENOTCONV))
    ctx.resume(snap)
    ctx.solve_step(60)
    x_resumed, _ = ctx.solve_finish(allow=(WF_OK, WF_ENOTCONV))
    assert np.array_equal(x_direct, x_resumed)
    # and equal to an uninterrupted 100-iteration solve
    x100, _ = ctx.solve(precision="fp64", tol=0.0, max_iter=100, allow=(WF_ENOTCONV,))
    assert np.array_equal(x100, x_direct)


def test_repeat_solves_bitwise_identical(ctx, pl32):
    _load(ctx, pl32)
    a, _ = ctx.solve(precision="mixed", tol=1e-9, max_iter=5000)
    b, _ = ctx.solve(precision="mixed", tol=1e-9, max_iter=5000)
    assert np.array_equal(a, b)


def test_mixed_snapshot_resume_bit_identical(pl32):
    """A mixed-precision solve stepped, snapshotted (FP64 x, r; FP32 x, r, p;
    scalars) and resumed in a new context continues bit for bit, and equals an
    uninterrupted mixed solve of as many FP32 iterations."""
    a = context()
    _load(a, pl32)
    a.solve_begin(precision="mixed", tol=1e-12, max_iter=100000)
    a.solve_step(45)
    snap = a.snapshot()
    a.solve_step(75)
    x_direct, info_d = a.solve_finish(allow=(WF_OK, WF_ENOTCONV))
    assert info_d.iters_total == 120 and info_d.outer_steps >= 2
    b = context()
    _load(b, pl32)
    b.resume(snap)
    b.solve_step(75)
    x_resumed, info_r = b.solve_finish(allow=(WF_OK, WF_ENOTCONV))
    assert np.array_equal(x_direct, x_resumed)
    assert info_r.outer_steps == info_d.outer_steps
    x120, info_u = a.solve(precision="mixed", tol=1e-12, max_iter=120, allow=(WF_ENOTCONV,))
    assert info_u.iters_total == 120
    assert np.array_equal(x120, x_direct)
    # the mixed snapshot holds two FP64 and three FP32 vectors (28 bytes per
    # cell), the FP64 one three FP64 vectors (24)
    a.solve_begin(precision="fp64", tol=1e-12, max_iter=100)
    a.solve_step(2)
    s64 = a.snapshot().size
    assert snap.size - s64 == 4 * 32 ** 3
    a.close()
    b.close()


def test_mixed_solve_reports_stagnation(pl32):
    """A mixed solve asked for a residual below what FP32 iterations with FP64
    updates reach stops as stagnated (WF_ENOTCONV) instead of running to
    max_iter, and its result is as good as the arithmetic allows."""
    ctx = context()
    _load(ctx, pl32)
    x, info = ctx.solve(precision="mixed", tol=1e-17, max_iter=100000, allow=(WF_ENOTCONV,))
    print(f"tol 1e-17: {info.iters_total} iterations, {info.outer_steps} updates, "
          f"residual {info.rel_res_true:.2e}, stagnated {info.stagnated}")
    assert info.status == WF_ENOTCONV and info.stagnated == 1
    assert info.iters_total < 5000
    assert info.rel_res_true < 1e-13
    assert rel_l2(x, pl32["x_ref"]) < 1e-9
    _, ok = ctx.solve(precision="mixed", tol=1e-10, max_iter=100000)
    assert ok.status == WF_OK and ok.stagnated == 0
    ctx.close()
