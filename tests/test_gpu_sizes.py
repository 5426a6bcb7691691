"""GPU parity at the grid sizes of the large workloads, against the oracle
(through the C ABI): the FFT passes at 192, 256, 384 and 512 in FP64 and FP32
(the 1024-thread FP32 tiles of grids from 256 up included), the plain
operator (eq:WF) at 256 and 384, the prior-split CG at 256 and 384 for a few
fixed iterations, and the supersampled deposit (Sec. 3.1.2) of a 384^3 grid,
whose fine 768^3 FFT and crop no smaller test reaches, at sampled nodes and
cells.  The oracle side uses scipy's multi-threaded FFT (the same transform
as numpy's)."""
import os

import numpy as np
import pytest

import synth
from oracle import deposit as od
from oracle import supersample as oss
from oracle import wiener as ow

from gpu_util import context, rel_l2, rel_max

pytestmark = pytest.mark.gpu

WORKERS = min(16, os.cpu_count() or 1)
WF_ENOTCONV = 5


@pytest.fixture(scope="module")
def ctx():
    c = context()
    yield c
    c.close()


def _rfftn(v):
    import scipy.fft as sf
    return sf.rfftn(v, workers=WORKERS)


@pytest.mark.parametrize("n", [192, 256, 384, 512])
def test_forward_spectrum_fp64_large(ctx, n):
    ctx.set_grid(n, 500.0)
    v = np.random.Generator(np.random.PCG64(n + 5)).standard_normal((n, n, n))
    got = ctx.forward_spectrum(v, "fp64")
    err = rel_max(got, _rfftn(v))
    print(f"fp64 forward {n}^3: max rel {err:.2e}")
    assert err < 1e-13 * np.log2(n)


@pytest.mark.parametrize("n", [192, 256, 384, 512])
def test_forward_spectrum_fp32_large(ctx, n):
    """FP32 passes on the FP32-rounded input; the bound grows with the number
    of butterfly stages (log2 n per axis) at ~1e-7 per stage."""
    ctx.set_grid(n, 500.0)
    v = np.random.Generator(np.random.PCG64(n + 6)).standard_normal((n, n, n))
    got = ctx.forward_spectrum(v, "mixed")
    err = rel_max(got, _rfftn(v.astype(np.float32).astype(np.float64)))
    print(f"fp32 forward {n}^3: max rel {err:.2e}")
    assert err < 3e-7 * np.log2(n)


def _random_system(ctx, n, box, seed):
    """A BBKS prior, a random mask with 30 % empty cells and a random RHS on
    the observed cells, loaded into the context and built in the oracle."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ptab = synth.p_by_m2(lambda k: synth.bbks_power(k), n, box)
    w = rng.uniform(0.05, 1.0, size=(n, n, n))
    w[rng.uniform(size=w.shape) < 0.3] = 0.0
    nbar = 0.61
    b = np.where(w > 0, rng.standard_normal((n, n, n)), 0.0)
    ctx.set_grid(n, box)
    ctx.set_mask(w)
    ctx.set_power(ptab)
    ctx.set_rhs(b, nbar)
    return ow.System(n, box, w, ptab, nbar, workers=WORKERS), b, rng


@pytest.mark.parametrize("n", [256, 384])
def test_operator_large(ctx, n):
    sysm, _, rng = _random_system(ctx, n, 500.0, n + 11)
    v = rng.standard_normal((n, n, n))
    ref = sysm.apply(v)
    e64 = rel_max(ctx.apply_operator(v, "fp64"), ref)
    v32 = v.astype(np.float32).astype(np.float64)
    e32 = rel_max(ctx.apply_operator(v32, "mixed"), sysm.apply(v32))
    print(f"operator {n}^3: fp64 {e64:.2e} fp32 {e32:.2e}")
    assert e64 < 1e-12
    assert e32 < 1e-5


@pytest.mark.parametrize("n", [256, 384])
def test_split_fixed_iterations_large(ctx, n):
    """Two CG iterations on the prior-split system from y = 0 (FP64 and
    mixed) against the oracle's split_cg: covers the direction-update x
    inverse, the z middle pass and the x forward pass with q at these sizes."""
    sysm, b, _ = _random_system(ctx, n, 500.0, n + 12)
    k = 2
    ref = ow.split_cg(sysm, b, 0.0, k)
    x, info = ctx.solve(precision="fp64", precond="prior", tol=0.0, max_iter=k,
                        allow=(WF_ENOTCONV,))
    assert info.iters_total == k
    e64 = rel_l2(x, ref["x"])
    y, info = ctx.solve(precision="mixed", precond="prior", tol=0.0, max_iter=k,
                        allow=(WF_ENOTCONV,))
    assert info.iters_total == k
    e32 = rel_l2(y, ref["x"])
    print(f"split k={k} {n}^3: fp64 {e64:.2e} mixed {e32:.2e}")
    assert e64 < 1e-12
    assert e32 < 1e-5


@pytest.mark.parametrize("n,scheme", [(192, "tsc"), (384, "cic")])
def test_supersampled_deposit_sampled(ctx, n, scheme):
    """The 2x deposit of an n^3 serving-size request (fine grid 2n): the int64
    grid bit for bit at the stencil nodes of 1500 galaxies and 3000 random
    nodes against the oracle's node-by-node evaluation, the exact total mass,
    and n^o at 40 cells against the oracle's direct summation (no FFT)."""
    import torch
    import paper_0906_3978_amd as wf
    wl = synth.Workload(f"s{n}", n, 500.0, scheme, 2, 400_000, 5200 + n, "bbks",
                        theta_deg=75.0, r0=180.0, axis=(0.6, 0.0, 0.8))
    ptab = wl.ptab()
    w = wl.mask()
    xyz = wl.catalogue(ptab, w).xyz
    ctx.set_grid(n, wl.box)
    ctx.set_mask(w)
    ctx.set_power(ptab)
    ctx.set_galaxies(xyz)
    ctx.deposit(scheme, 2)
    nf = 2 * n
    g = torch.empty((nf, nf, nf), dtype=torch.int64, device="cuda:0")
    nobs = torch.empty((n, n, n), dtype=torch.float64, device="cuda:0")
    assert wf.lib().wf_get_deposit(ctx._h, g.data_ptr(), nobs.data_ptr(), None, 1) == 0
    torch.cuda.synchronize()
    assert int(g.sum().item()) == len(xyz) * (1 << 39)
    rng = np.random.Generator(np.random.PCG64(n))
    pick = xyz[rng.choice(len(xyz), 1500, replace=False)]
    near = np.floor(pick * (nf / wl.box) + 0.5).astype(np.int64)
    offs = np.array([(i, j, k) for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)])
    nodes = (near[:, None, :] + offs[None, :, :]).reshape(-1, 3) % nf
    nodes = np.unique(np.concatenate([nodes, rng.integers(0, nf, size=(3000, 3))]), axis=0)
    flat = (nodes[:, 0] * nf + nodes[:, 1]) * nf + nodes[:, 2]
    got = g.view(-1)[torch.from_numpy(flat).to(g.device)].cpu().numpy()
    assert np.array_equal(got, od.deposit_at(xyz, nf, wl.box, scheme, nodes))
    del g
    cells = np.concatenate([np.floor(pick[:20] * (n / wl.box) + 0.5).astype(np.int64) % n,
                            rng.integers(0, n, size=(20, 3))])
    cflat = (cells[:, 0] * n + cells[:, 1]) * n + cells[:, 2]
    got_c = nobs.view(-1)[torch.from_numpy(cflat).to(nobs.device)].cpu().numpy()
    want = oss.observed_counts_at(xyz, n, wl.box, scheme, cells)
    err = np.abs(got_c - want).max() / np.abs(want).max()
    print(f"{nf}^3 {scheme} deposit: {len(nodes)} nodes; n_obs at 40 cells max rel {err:.2e}")
    assert err <= 1e-11
    # the low-passed field keeps the mass: sum n^o = N_gal
    assert float(nobs.sum().item()) == pytest.approx(len(xyz), rel=1e-12)
