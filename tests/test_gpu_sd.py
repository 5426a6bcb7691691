"""GPU parity of the signal-dependent noise formulation (eq:noisecov, Sec. 3.4)
against the oracle, through the C ABI: jackknife thinning (bit-exact counts),
the mean-estimator solve and jackknife batches."""
import numpy as np
import pytest

import synth
from oracle import sdnoise as sd
from oracle import supersample as oss
from oracle import wiener as ow

from gpu_util import context, rel_l2

pytestmark = pytest.mark.gpu

WF_OK, WF_ENOTCONV = 0, 5
SEED = 0x1234_5678_9ABC_DEF0


@pytest.fixture(scope="module")
def ctx():
    c = context()
    yield c
    c.close()


def _workload(n, box, ngal, seed, scheme="cic", ss=2):
    wl = synth.Workload(f"sd{n}", n, box, scheme, ss, ngal, seed, "bbks")
    ptab = wl.ptab()
    w = wl.mask()
    xyz = wl.catalogue(ptab, w).xyz
    nobs, _ = oss.observed_counts(xyz, n, box, scheme, ss)
    nbar = ow.mean_density(len(xyz), w)
    alpha = 0.9 * float(w[w > 0].min())
    return dict(wl=wl, ptab=ptab, w=w, xyz=xyz, nobs=nobs, nbar=nbar, alpha=alpha)


def _load(ctx, d):
    wl = d["wl"]
    ctx.set_grid(wl.n, wl.box)
    ctx.set_mask(d["w"])
    ctx.set_power(d["ptab"])
    ctx.set_galaxies(d["xyz"])
    ctx.deposit(wl.scheme, wl.supersample)


def _oracle_system(d, kind, j=0, seed=SEED):
    wl = d["wl"]
    if kind == "mean":
        lam = sd.lambda_obs_mean(sd.ngp_counts(d["xyz"], wl.n, wl.box, d["w"]))
    else:
        t = sd.thinned_counts(d["xyz"], wl.n, wl.box, d["w"], d["alpha"], seed, j)
        lam = sd.lambda_obs_jackknife(t, d["w"], d["alpha"])
    sysm = sd.SDSystem(wl.n, wl.box, d["w"], d["ptab"], d["nbar"], lam)
    return sysm, sysm.data_vector(d["nobs"])


@pytest.fixture(scope="module")
def sd32():
    return _workload(32, 300.0, 30000, 601)


def test_jackknife_counts_bit_exact(ctx, sd32):
    d = sd32
    wl = d["wl"]
    ctx.set_grid(wl.n, wl.box)
    ctx.set_mask(d["w"])
    ctx.set_galaxies(d["xyz"])
    for first, count in [(0, 4), ((1 << 32) + 3, 2)]:
        got = ctx.jackknife_counts(d["alpha"], SEED, first, count)
        for j in range(count):
            want = sd.thinned_counts(d["xyz"], wl.n, wl.box, d["w"], d["alpha"], SEED, first + j)
            assert np.array_equal(got[j], want)
    # keep probability one on every node where w = alpha: all galaxies kept
    full = sd.ngp_counts(d["xyz"], wl.n, wl.box, d["w"])
    assert got[0].sum() < full.sum()


def test_jackknife_rejects_large_alpha(ctx, sd32):
    import paper_0906_3978_amd as wf
    d = sd32
    ctx.set_grid(d["wl"].n, d["wl"].box)
    ctx.set_mask(d["w"])
    ctx.set_galaxies(d["xyz"])
    with pytest.raises(wf.WienerError):
        ctx.jackknife_counts(1.01 * float(d["w"].max()), 1, 0, 1)


def test_sd_needs_a_current_deposit(ctx, sd32):
    import paper_0906_3978_amd as wf
    d = sd32
    _load(ctx, d)
    ctx.set_galaxies(d["xyz"])
    with pytest.raises(wf.WienerError):
        ctx.solve_sd("mean", precision="fp64", tol=1e-8)


@pytest.mark.parametrize("k", [1, 30])
def test_sd_mean_fixed_iterations(ctx, sd32, k):
    """k CG iterations on the SD system (plain CG, FP64) on both sides."""
    d = sd32
    _load(ctx, d)
    x, _, infos = ctx.solve_sd("mean", precision="fp64", tol=0.0, max_iter=k,
                               allow=(WF_ENOTCONV,))
    assert infos[0].iters_total == k
    sysm, b = _oracle_system(d, "mean")
    ref = ow.cg(sysm, b, 0.0, k)
    err = rel_l2(x, ref["x"])
    print(f"sd mean k={k}: rel_l2 {err:.3e}")
    # the oracle perturbed by 1e-16 per application moves by 6e-16 at k = 30
    assert err < (1e-13 if k == 1 else 1e-11)
    assert abs(infos[0].rel_res_recursive - ref["rel_res"]) < 1e-10


@pytest.mark.parametrize("precond", ["none", "prior"])
def test_sd_mean_converged(ctx, sd32, precond):
    d = sd32
    _load(ctx, d)
    x, _, infos = ctx.solve_sd("mean", precision="fp64", precond=precond, tol=1e-12,
                               max_iter=20000)
    assert infos[0].status == WF_OK
    sysm, b = _oracle_system(d, "mean")
    ref = ow.split_cg(sysm, b, 1e-13, 20000)
    err = rel_l2(x, ref["x"])
    print(f"sd mean {precond}: iters {infos[0].iters_total} rel_l2 {err:.3e}")
    assert err < 1e-9
    # the SD solution differs from the LSQ one (the noise model matters)
    y, _ = ctx.solve(precision="fp64", precond=precond, tol=1e-12, max_iter=20000)
    assert rel_l2(x, y) > 1e-3


def test_sd_jackknife_batch_fp64():
    """18 samples at 16^3: one batch of 16 and one of 2; every sample and the
    mean against the oracle."""
    d = _workload(16, 200.0, 6000, 602)
    ctx = context()
    _load(ctx, d)
    mean, xs, infos = ctx.solve_sd("jackknife", alpha=d["alpha"], seed=SEED, first=7,
                                   nsamples=18, keep_samples=True, precision="fp64",
                                   precond="prior", tol=1e-12, max_iter=20000)
    assert all(i.status == WF_OK for i in infos)
    refs = []
    for j in range(18):
        sysm, b = _oracle_system(d, "jackknife", 7 + j)
        refs.append(ow.split_cg(sysm, b, 1e-13, 20000)["x"])
        assert rel_l2(xs[j], refs[-1]) < 1e-9
    assert rel_l2(mean, np.mean(refs, axis=0)) < 1e-9
    assert np.array_equal(mean, xs.sum(axis=0) / 18) or rel_l2(mean, xs.mean(axis=0)) < 1e-15
    # a sample solved alone gives the same bits as inside the batch
    one, _, _ = ctx.solve_sd("jackknife", alpha=d["alpha"], seed=SEED, first=7 + 16, nsamples=1,
                             precision="fp64", precond="prior", tol=1e-12, max_iter=20000)
    assert np.array_equal(one, xs[16])
    ctx.close()


@pytest.mark.parametrize("tol", [1e-6, 1e-9])
def test_sd_jackknife_mixed(ctx, sd32, tol):
    d = sd32
    _load(ctx, d)
    mean, xs, infos = ctx.solve_sd("jackknife", alpha=d["alpha"], seed=SEED, nsamples=3,
                                   keep_samples=True, precision="mixed", precond="prior",
                                   tol=tol, max_iter=20000)
    for j in range(3):
        assert infos[j].status == WF_OK
        sysm, b = _oracle_system(d, "jackknife", j)
        ref = ow.split_cg(sysm, b, 1e-13, 20000)["x"]
        sp = ow.SplitSystem(sysm)
        r = sp.split(b - sysm.apply(xs[j]))
        rel = float(np.linalg.norm(r) / np.linalg.norm(sp.split(b)))
        err = rel_l2(xs[j], ref)
        print(f"sd jk mixed tol={tol:g} j={j}: iters {infos[j].iters_total} split res "
              f"{rel:.3e} err {err:.3e}")
        assert rel <= 1.01 * tol
        assert err < 300 * tol
        # batch == single
        one, _, _ = ctx.solve_sd("jackknife", alpha=d["alpha"], seed=SEED, first=j, nsamples=1,
                                 precision="mixed", precond="prior", tol=tol, max_iter=20000)
        assert np.array_equal(one, xs[j])


def test_sd_without_galaxies_is_zero(ctx, sd32):
    """No galaxies: nbar = 0, so the noise diagonals and the data vanish and
    every sample's solution is zero (no iteration needed)."""
    d = sd32
    wl = d["wl"]
    ctx.set_grid(wl.n, wl.box)
    ctx.set_mask(d["w"])
    ctx.set_power(d["ptab"])
    ctx.set_galaxies(np.zeros((0, 3)))
    ctx.deposit("cic", 2)
    for kind, ns in (("mean", 1), ("jackknife", 3)):
        mean, xs, infos = ctx.solve_sd(kind, alpha=d["alpha"], seed=1, nsamples=ns,
                                       keep_samples=True, precision="mixed", precond="prior",
                                       tol=1e-8, max_iter=100)
        assert not mean.any() and not xs.any()
        assert all(i.status == WF_OK and i.iters_total == 0 for i in infos)


def test_sd_and_post_with_device_buffers(ctx, sd32):
    """The same calls with device (torch) buffers give the host-buffer results
    bit for bit."""
    import torch
    d = sd32
    _load(ctx, d)
    kw = dict(precision="mixed", precond="prior", tol=1e-8, max_iter=20000)
    mean_h, xs_h, _ = ctx.solve_sd("jackknife", alpha=d["alpha"], seed=3, nsamples=2,
                                   keep_samples=True, **kw)
    dev = torch.device("cuda:0")
    mean_d = torch.empty(mean_h.shape, dtype=torch.float64, device=dev)
    _, xs_d, _ = ctx.solve_sd("jackknife", alpha=d["alpha"], seed=3, nsamples=2,
                              mean_out=mean_d, keep_samples=True, **kw)
    assert np.array_equal(mean_d.cpu().numpy(), mean_h)
    assert np.array_equal(xs_d.cpu().numpy(), xs_h)
    sm_h = ctx.fourier_filter(mean_h, "gauss", a=6.0)
    sm_d = ctx.fourier_filter(mean_d, "gauss", a=6.0)
    assert np.array_equal(sm_d.cpu().numpy(), sm_h)
    assert ctx.field_moments(sm_d, masked=True) == ctx.field_moments(sm_h, masked=True)
    assert np.array_equal(ctx.compare_fields(sm_d, mean_d), ctx.compare_fields(sm_h, mean_h),
                          equal_nan=True)
