"""GPU parity of the prior-split CG, (C A C) y = C b with s = C y (C the square
root of the prior covariance, Sec. 3.3.1), against the oracle's split_cg,
through the C ABI."""
import numpy as np
import pytest

import synth
from oracle import wiener as ow

from gpu_util import context, rel_l2
import sensitivity as se

pytestmark = pytest.mark.gpu

WF_OK, WF_EINVAL, WF_ENOTCONV = 0, 1, 5


@pytest.fixture(scope="module")
def ctx():
    c = context()
    yield c
    c.close()


@pytest.fixture(scope="module")
def bbks48():
    """48^3 / 500 Mpc, BBKS prior, cap mask, lognormal-Poisson catalogue,
    2x supersampled CIC (the plain solver's fixed-k parity workload)."""
    wl = synth.Workload("bbks48", 48, 500.0, "cic", 2, 60000, 211, "bbks")
    ptab = wl.ptab()
    w = wl.mask()
    cat = wl.catalogue(ptab, w)
    res = ow.reconstruct(cat.xyz, wl.n, wl.box, w, ptab, "cic", 2, 1e-10, 5000)
    ref = ow.reference_solution(res["system"], res["b"], tol=1e-13)
    return dict(wl=wl, ptab=ptab, w=w, xyz=cat.xyz, res=res, x_ref=ref["x"])


def _load(ctx, d):
    wl = d["wl"]
    ctx.set_grid(wl.n, wl.box)
    ctx.set_mask(d["w"])
    ctx.set_power(d["ptab"])
    ctx.set_galaxies(d["xyz"])
    ctx.deposit("cic", 2)


@pytest.mark.parametrize("k", [1, 20, 80, 200])
def test_fixed_iteration_parity_split_fp64(ctx, bbks48, k):
    """Both sides run exactly k iterations of CG on C A C from y = 0.  The
    bound is a multiple of the oracle's own spread at that k under
    rounding-sized noise (tests/sensitivity.py): its iterates move by 2e-9
    at k = 20, 2.4e-8 at k = 80 (the phase where the large eigenvalues are
    being resolved) and 5e-14 at k = 200."""
    tol = se.bound("bbks48", "split", k)
    d = bbks48
    _load(ctx, d)
    x, info = ctx.solve(precision="fp64", precond="prior", tol=0.0, max_iter=k,
                        allow=(WF_ENOTCONV,))
    assert info.iters_total == k and info.status == WF_ENOTCONV
    ref = ow.split_cg(d["res"]["system"], d["res"]["b"], 0.0, k)
    err = rel_l2(x, ref["x"])
    print(f"split fixed k={k}: rel_l2 {err:.3e} bound {tol:.1e} "
          f"({err / max(se.SPREADS[('bbks48', 'split', k)], 1e-300):.2f} x the oracle's spread) "
          f"rec {info.rel_res_recursive:.6e} vs {ref['rel_res']:.6e}")
    assert err < tol
    # residuals relative to ||C b|| and ||b||: their spread follows the iterates'
    assert abs(info.rel_res_recursive - ref["rel_res"]) < max(1e-12, tol)
    assert abs(info.rel_res_true - ref["rel_res_true"]) < max(1e-12, tol)


def test_split_converged_fp64(ctx, bbks48):
    d = bbks48
    _load(ctx, d)
    x, info = ctx.solve(precision="fp64", precond="prior", tol=1e-12, max_iter=5000)
    assert info.status == WF_OK
    assert info.rel_res_recursive <= 1e-12
    assert rel_l2(x, d["x_ref"]) < 1e-10
    assert info.rel_res_true < 1e-9


def test_split_needs_fewer_iterations(ctx, bbks48):
    d = bbks48
    _load(ctx, d)
    _, plain = ctx.solve(precision="fp64", tol=1e-8, max_iter=20000)
    x, split = ctx.solve(precision="fp64", precond="prior", tol=1e-8, max_iter=20000)
    print(f"iterations to 1e-8: plain {plain.iters_total} split {split.iters_total}")
    assert split.iters_total < plain.iters_total
    assert rel_l2(x, d["x_ref"]) < 1e-6


@pytest.mark.parametrize("tol", [1e-7, 1e-10])
def test_split_mixed(ctx, bbks48, tol):
    """FP32 operator and vectors with FP64 reliable updates on the split
    system; convergence is decided on the FP64 split residual."""
    d = bbks48
    _load(ctx, d)
    x, info = ctx.solve(precision="mixed", precond="prior", tol=tol, max_iter=20000)
    assert info.status == WF_OK
    assert info.outer_steps >= 1
    err = rel_l2(x, d["x_ref"])
    # the oracle recomputes the split residual ||C (b - A s)|| / ||C b|| of the
    # returned solution: the device stopped on the same quantity in FP64
    sysm = d["res"]["system"]
    b = d["res"]["b"]
    sp = ow.SplitSystem(sysm)
    r = sp.split(b - sysm.apply(x))
    rel = float(np.linalg.norm(r) / np.linalg.norm(sp.split(b)))
    print(f"split mixed tol={tol:g}: iters {info.iters_total} updates {info.outer_steps} "
          f"split res {rel:.3e} err {err:.3e} true res {info.rel_res_true:.3e}")
    assert rel <= 1.01 * tol
    # error per unit of split residual on this workload: ~2 early, ~120 once the
    # small-scale modes dominate what is left (FP64 reaches 1e-12 -> err < 1e-10)
    assert err < 300 * tol
    # the same solve twice gives the same bits
    y, _ = ctx.solve(precision="mixed", precond="prior", tol=tol, max_iter=20000)
    assert np.array_equal(x, y)


@pytest.mark.parametrize("precond", ["prior", "none"])
def test_mixed_last_change_is_the_change_of_s(ctx, bbks48, precond):
    """The change a reliable update reports (last_change, what the settle rule
    sums) is ||s_k+1 - s_k|| / ||s_k+1|| of the solutions the same mixed solve
    returns when it is stopped after k and after k + 1 updates (the two runs
    agree bit for bit up to the k-th).  The prior-split form measures it on
    the half spectrum of y, each mode weighted by its factor squared: this
    pins that weighting to the modes' places in the vectors' tile layout (the
    weights of the [x][y][kz] order instead, which the vectors do not use,
    put the value several per cent off here).  The bound: in the kz = 0 and N/2
    planes the half spectrum stores both members of each conjugate pair, and
    the FP32 iteration leaves them conjugate only to rounding; that part has
    no real-space counterpart and adds ~(1e-7 ||y|| / ||change||)^2 / 2 to the
    reported value, 3e-7 of it for a change of 1e-4 (measured at update 5)."""
    _load(ctx, bbks48)
    kw = dict(precision="mixed", precond=precond, tol=1e-14, max_iter=100000, err_tol=-1.0,
              allow=(WF_ENOTCONV,))
    for k in (2, 4):
        xa, ia = ctx.solve(max_outer=k, **kw)
        xb, ib = ctx.solve(max_outer=k + 1, **kw)
        assert ib.outer_steps == ia.outer_steps + 1 and ib.iters_total > ia.iters_total
        change = float(np.linalg.norm(xb - xa) / np.linalg.norm(xb))
        print(f"{precond} update {k + 1}: reported {ib.last_change:.6e}, "
              f"from the solutions {change:.6e}")
        assert 1e-8 < change < 1.0
        assert abs(ib.last_change / change - 1.0) < 1e-5


def test_split_zero_rhs(ctx, bbks48):
    d = bbks48
    wl = d["wl"]
    ctx.set_grid(wl.n, wl.box)
    ctx.set_mask(d["w"])
    ctx.set_power(d["ptab"])
    ctx.set_rhs(np.zeros((wl.n,) * 3), 1.0)
    for prec in ("fp64", "mixed"):
        x, info = ctx.solve(precision=prec, precond="prior", tol=1e-10, max_iter=100)
        assert info.status == WF_OK and info.iters_total == 0
        assert not x.any()


def test_split_batch_equals_single():
    wl = synth.Workload("b32", 32, 300.0, "cic", 2, 30000, 401, "bbks")
    ptab = wl.ptab()
    w = wl.mask()
    cats = []
    for j in range(3):
        wl.seed = 401 + 3 * j
        cats.append(wl.catalogue(ptab, w).xyz)
    ctx = context()
    ctx.set_grid(wl.n, wl.box)
    ctx.set_mask(w)
    ctx.set_power(ptab)
    for prec in ("mixed", "fp64"):
        outs, infos = ctx.solve_batch(cats, "cic", 2, precision=prec, precond="prior", tol=1e-9,
                                      max_iter=20000)
        for xyz, x, info in zip(cats, outs, infos):
            assert info.status == WF_OK
            ctx.set_galaxies(xyz)
            ctx.deposit("cic", 2)
            y, inf1 = ctx.solve(precision=prec, precond="prior", tol=1e-9, max_iter=20000)
            assert np.array_equal(x, y)
            assert info.iters_total == inf1.iters_total
    res = ow.reconstruct(cats[1], wl.n, wl.box, w, ptab, "cic", 2, 1e-12, 20000)
    assert rel_l2(outs[1], res["x"]) < 1e-6
    ctx.close()


def test_split_server_equals_context():
    import paper_0906_3978_amd as wf
    reqs = []
    for i, n in enumerate([16, 32, 24]):
        wl = synth.serving_request(i, base_seed=950, box=300.0, grids=(n,))
        wl.n_target = min(wl.n_target, 30000)
        ptab = wl.ptab()
        w = wl.mask()
        reqs.append((wl, ptab, w, wl.catalogue(ptab, w).xyz))
    kw = dict(precision="mixed", precond="prior", tol=1e-9, max_iter=20000)
    with wf.Server(0, hbm_budget=1 << 30, max_active=4) as srv:
        tickets = [srv.submit(wl.n, wl.box, w, p, xyz, "cic", 2, **kw) for wl, p, w, xyz in reqs]
        got = [srv.wait(t, wl.n) for t, (wl, _, _, _) in zip(tickets, reqs)]
    ctx = context()
    for (wl, p, w, xyz), (x, info) in zip(reqs, got):
        assert info.status == WF_OK
        ctx.set_grid(wl.n, wl.box)
        ctx.set_mask(w)
        ctx.set_power(p)
        ctx.set_galaxies(xyz)
        ctx.deposit("cic", 2)
        y, inf1 = ctx.solve(**kw)
        assert np.array_equal(x, y)
        assert info.iters_total == inf1.iters_total
    ctx.close()


def test_split_option_checks(ctx, bbks48):
    import ctypes
    import paper_0906_3978_amd as wf
    _load(ctx, bbks48)
    o = wf.opts(precision="fp64", tol=1e-8)
    o.precond = 7
    L = wf.lib()
    out = np.empty((48,) * 3)
    assert L.wf_solve(ctx._h, ctypes.byref(o), out.ctypes.data, 0, None) == WF_EINVAL
    o = wf.opts(precision="mixed", tol=1e-8, precond="prior")
    o.err_tol = float("nan")
    assert L.wf_solve(ctx._h, ctypes.byref(o), out.ctypes.data, 0, None) == WF_EINVAL
    with pytest.raises(wf.WienerError):
        ctx.solve_begin(precision="mixed", precond="prior", tol=-1.0)


@pytest.mark.parametrize("n", [8, 12, 16, 24, 64, 96])
def test_split_across_grid_sizes(ctx, n):
    """Converged prior-split solves (FP64 and mixed) on grids whose FFT plans
    differ (radix 2, 3, 4, 8 mixes; tiles narrower than the default), against
    the oracle's split CG."""
    wl = synth.Workload(f"g{n}", n, 4.0 * n, "cic", 2, 40 * n ** 2, 700 + n, "bbks")
    ptab = wl.ptab()
    w = wl.mask()
    xyz = wl.catalogue(ptab, w).xyz
    res = ow.reconstruct(xyz, n, wl.box, w, ptab, "cic", 2, 1e-10, 5000)
    ref = ow.split_cg(res["system"], res["b"], 1e-13, 20000)["x"]
    ctx.set_grid(n, wl.box)
    ctx.set_mask(w)
    ctx.set_power(ptab)
    ctx.set_galaxies(xyz)
    ctx.deposit("cic", 2)
    x, info = ctx.solve(precision="fp64", precond="prior", tol=1e-12, max_iter=20000)
    assert info.status == WF_OK
    assert rel_l2(x, ref) < 1e-9
    y, info = ctx.solve(precision="mixed", precond="prior", tol=1e-9, max_iter=20000)
    assert info.status == WF_OK
    assert rel_l2(y, ref) < 300 * 1e-9


def test_split_snapshot_resume_bit_identical(bbks48):
    """The stepwise FP64 prior-split solve: a snapshot resumed in a new
    context continues bit for bit, and equals an uninterrupted solve of as
    many iterations."""
    d = bbks48
    a = context()
    _load(a, d)
    a.solve_begin(precision="fp64", precond="prior", tol=1e-12, max_iter=5000)
    a.solve_step(25)
    snap = a.snapshot()
    a.solve_step(35)
    x_direct, info_d = a.solve_finish(allow=(WF_OK, WF_ENOTCONV))
    assert info_d.iters_total == 60
    b = context()
    _load(b, d)
    b.resume(snap)
    b.solve_step(35)
    x_resumed, info_r = b.solve_finish(allow=(WF_OK, WF_ENOTCONV))
    assert np.array_equal(x_direct, x_resumed)
    assert info_r.rel_res_true == info_d.rel_res_true
    x60, _ = a.solve(precision="fp64", precond="prior", tol=0.0, max_iter=60,
                     allow=(WF_ENOTCONV,))
    assert np.array_equal(x60, x_direct)
    # a plain snapshot is smaller and resumes as a plain solve
    a.solve_begin(precision="fp64", tol=1e-12, max_iter=5000)
    a.solve_step(5)
    assert a.snapshot().size < snap.size
    a.close()
    b.close()


def test_split_mixed_snapshot_resume_bit_identical(bbks48):
    """The same for a mixed prior-split solve, whose snapshot holds half
    spectra and whose resumed updates recompute C b from the data."""
    d = bbks48
    a = context()
    _load(a, d)
    a.solve_begin(precision="mixed", precond="prior", tol=1e-12, max_iter=100000)
    a.solve_step(30)
    snap = a.snapshot()
    a.solve_step(50)
    x_direct, info_d = a.solve_finish(allow=(WF_OK, WF_ENOTCONV))
    assert info_d.iters_total == 80
    b = context()
    _load(b, d)
    b.resume(snap)
    b.solve_step(50)
    x_resumed, _ = b.solve_finish(allow=(WF_OK, WF_ENOTCONV))
    assert np.array_equal(x_direct, x_resumed)
    x80, _ = a.solve(precision="mixed", precond="prior", tol=1e-12, max_iter=80,
                     allow=(WF_ENOTCONV,))
    assert np.array_equal(x80, x_direct)
    a.close()
    b.close()
