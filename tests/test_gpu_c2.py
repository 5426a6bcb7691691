"""The 256^3 plain FP64 workload (BBKS prior, 500 Mpc box, 60 deg cap with
exp(-r/150 Mpc), 1e6 lognormal-Poisson galaxies, CIC on the 2x grid, CG to a
relative residual of 1e-6) at full size, against oracle references stored at
every 8th cell along each axis by tests/golden/make_fixed_k.py (which calls
only the oracle): the deposit and n^o, exactly k = 50 and k = 300 CG
iterations, and the solve stopped at 1e-6 compared with the oracle stopped at
the same residual (eq:WF, Sec. 3.3.1; gridding per Sec. 3.1.2)."""
import json
import os

import numpy as np
import pytest

import synth

from gpu_util import context
import sensitivity as se

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
WF_OK, WF_ENOTCONV = 0, 5


@pytest.fixture(scope="module")
def c2():
    stem = os.path.join(GOLDEN, "bbks256_n256_cg")
    with open(stem + ".json") as fh:
        meta = json.load(fh)
    ref = dict(np.load(stem + ".npz"))
    wl = synth.workload("bbks256")
    ptab = wl.ptab()
    w = wl.mask()
    cat = wl.catalogue(ptab, w)
    assert len(cat.xyz) == meta["n_gal"]
    ctx = context()
    ctx.set_grid(wl.n, wl.box)
    ctx.set_mask(w)
    ctx.set_power(ptab)
    ctx.set_galaxies(cat.xyz)
    ctx.deposit(wl.scheme, wl.supersample)
    yield dict(ctx=ctx, meta=meta, ref=ref, wl=wl, xyz=cat.xyz)
    ctx.close()


def _s(x, c2):
    st = c2["meta"]["stride"]
    return x[::st, ::st, ::st]


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_c2_deposit_and_data(c2):
    """n^o (low-pass of the 512^3 CIC grid) and b at the sampled cells, the
    integer total of the fine grid, and nbar, against the oracle's."""
    import torch
    import paper_0906_3978_amd as wf
    meta, ref = c2["meta"], c2["ref"]
    n = meta["n"]
    _, nobs, nbar = c2["ctx"].get_deposit(False, True, 2)
    assert nbar == pytest.approx(meta["nbar"], rel=1e-15)
    e = np.abs(_s(nobs, c2) - ref["n_obs"]).max() / np.abs(ref["n_obs"]).max()
    print(f"256^3 n_obs at {ref['n_obs'].size} cells: max rel {e:.2e}")
    assert e < 1e-13
    nf = 2 * n
    g = torch.empty((nf, nf, nf), dtype=torch.int64, device="cuda:0")
    assert wf.lib().wf_get_deposit(c2["ctx"]._h, g.data_ptr(), None, None, 1) == 0
    assert int(g.sum().item()) == meta["deposit_total"] == len(c2["xyz"]) << 39


def test_c2_fixed_50_iterations(c2):
    """Both sides run exactly 50 CG iterations from x = 0; the bound is a
    multiple of the oracle's own spread at k = 50 under rounding-sized noise
    (tests/sensitivity.py; measured by the script that wrote the reference)."""
    k = 50
    fk = c2["meta"]["fixed_k"][str(k)]
    x, info = c2["ctx"].solve(precision="fp64", tol=0.0, max_iter=k, allow=(WF_ENOTCONV,))
    assert info.iters_total == k
    err = _rel(_s(x, c2), c2["ref"][f"x_k{k}"])
    norm = abs(np.linalg.norm(x) / fk["x_norm"] - 1.0)
    bound = max(se.FACTOR * fk["spread"], se.FLOOR)
    print(f"256^3 k={k}: sampled rel L2 {err:.3e} |x| off {norm:.1e} (oracle spread "
          f"{fk['spread']:.2e}, bound {bound:.1e}); rec res {info.rel_res_recursive:.9e} vs "
          f"{fk['rel_res']:.9e}")
    assert err < bound
    assert norm < bound
    assert info.rel_res_recursive == pytest.approx(fk["rel_res"], rel=max(bound, 1e-9))


def test_c2_fixed_300_iterations(c2):
    """Exactly 300 CG iterations.  Here the iterates are chaotic under
    rounding: the oracle's own 300th iterate moves by 1.1e-5 under the
    rounding model and by 2.3e-5 under ten times that noise (it saturates), so
    no fixed-iterate bound near the survey's 1e-10 is meaningful.  What is
    fixed is how good the iterate is: it is 3.2e-2 from A^-1 b, and the GPU's
    must be as good (its distance from A^-1 b within 1 % of the oracle's) and
    differ from the oracle's by at most 1 % of that distance."""
    k = 300
    ref = c2["ref"]
    fk = c2["meta"]["fixed_k"][str(k)]
    x, info = c2["ctx"].solve(precision="fp64", tol=0.0, max_iter=k, allow=(WF_ENOTCONV,))
    assert info.iters_total == k
    xs = _s(x, c2)
    e_or = _rel(ref[f"x_k{k}"], ref["x_ref"])
    e_gpu = _rel(xs, ref["x_ref"])
    diff = _rel(xs, ref[f"x_k{k}"])
    print(f"256^3 k={k}: GPU - oracle {diff:.3e}; distance from A^-1 b: GPU {e_gpu:.4e}, "
          f"oracle {e_or:.4e}; oracle spread {fk['spread']:.2e}; rec res "
          f"{info.rel_res_recursive:.6e} vs {fk['rel_res']:.6e}")
    assert abs(e_gpu / e_or - 1.0) < 0.01
    assert diff < 0.01 * e_or
    assert info.rel_res_recursive == pytest.approx(fk["rel_res"], rel=0.05)


def test_c2_same_stop(c2):
    """CG stopped at ||r||/||b|| <= 1e-6: the GPU result is at most twice as
    far from A^-1 b as the oracle's result at the same stop (+1e-12), and
    takes the oracle's iteration count within 3."""
    meta, ref = c2["meta"], c2["ref"]
    tol = meta["stop"]["tol"]
    x, info = c2["ctx"].solve(precision="fp64", tol=tol, max_iter=100000)
    assert info.status == WF_OK
    e_gpu = _rel(_s(x, c2), ref["x_ref"])
    e_or = _rel(ref["x_tol"], ref["x_ref"])
    print(f"256^3 fp64 to {tol:g}: {info.iters_total} iterations (oracle "
          f"{meta['stop']['iterations']}), true res {info.rel_res_true:.3e}, sampled error "
          f"{e_gpu:.3e} vs oracle {e_or:.3e}")
    assert abs(info.iters_total - meta["stop"]["iterations"]) <= 3
    assert info.rel_res_true <= 1.05 * tol
    assert e_gpu <= 2 * e_or + 1e-12


@pytest.mark.parametrize("precond,tol", [("prior", 3e-7), ("none", 2e-9)])
def test_c2_mixed_error(c2, precond, tol):
    """The mixed-precision solves of the benchmark's tolerances stay within
    1e-6 relative L2 of the oracle's A^-1 b at the sampled cells."""
    ref = c2["ref"]
    x, info = c2["ctx"].solve(precision="mixed", precond=precond, tol=tol, max_iter=100000)
    assert info.status == WF_OK
    err = _rel(_s(x, c2), ref["x_ref"])
    print(f"256^3 mixed {precond} to {tol:g}: {info.iters_total} iterations, "
          f"{info.outer_steps} FP64 residuals, sampled error {err:.3e}")
    assert err < 1e-6
