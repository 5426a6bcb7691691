"""GPU parity of the FFT passes, the operator and the deposit against the
oracle (element by element, through the C ABI)."""
import numpy as np
import pytest

import synth
from oracle import deposit as od
from oracle import supersample as oss
from oracle import wiener as ow

from gpu_util import context, rel_max

pytestmark = pytest.mark.gpu

SIZES = [8, 12, 16, 24, 32, 48, 64, 96, 128]


@pytest.fixture(scope="module")
def ctx():
    c = context()
    yield c
    c.close()


@pytest.mark.parametrize("n", SIZES)
def test_forward_spectrum_fp64(ctx, n):
    ctx.set_grid(n, 100.0)
    v = np.random.Generator(np.random.PCG64(n)).standard_normal((n, n, n))
    got = ctx.forward_spectrum(v, "fp64")
    ref = np.fft.rfftn(v)
    assert rel_max(got, ref) < 1e-13 * np.log2(n)


@pytest.mark.parametrize("n", [8, 12, 32, 96, 128])
def test_forward_spectrum_fp32(ctx, n):
    ctx.set_grid(n, 100.0)
    v = np.random.Generator(np.random.PCG64(n)).standard_normal((n, n, n))
    got = ctx.forward_spectrum(v, "mixed")
    ref = np.fft.rfftn(v.astype(np.float32).astype(np.float64))
    assert rel_max(got, ref) < 2e-6


def _operator_setup(ctx, n, box, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    ptab = synth.p_by_m2(lambda k: synth.bbks_power(k), n, box)
    w = rng.uniform(0.05, 1.0, size=(n, n, n))
    w[rng.uniform(size=w.shape) < 0.3] = 0.0
    nbar = 0.83
    b = np.where(w > 0, rng.standard_normal((n, n, n)), 0.0)
    ctx.set_grid(n, box)
    ctx.set_mask(w)
    ctx.set_power(ptab)
    ctx.set_rhs(b, nbar)
    return ow.System(n, box, w, ptab, nbar), rng


@pytest.mark.parametrize("n", [8, 12, 24, 32, 48, 64])
def test_operator_fp64(ctx, n):
    sysm, rng = _operator_setup(ctx, n, 150.0, n + 1)
    v = rng.standard_normal((n, n, n))
    got = ctx.apply_operator(v, "fp64")
    ref = sysm.apply(v)
    assert rel_max(got, ref) < 1e-12


@pytest.mark.parametrize("n", [16, 48, 64])
def test_operator_fp32(ctx, n):
    sysm, rng = _operator_setup(ctx, n, 150.0, n + 2)
    v = rng.standard_normal((n, n, n))
    got = ctx.apply_operator(v, "mixed")
    ref = sysm.apply(v.astype(np.float32).astype(np.float64))
    assert rel_max(got, ref) < 1e-5


@pytest.mark.parametrize("scheme", ["ngp", "cic", "tsc"])
@pytest.mark.parametrize("n,ss", [(16, 1), (24, 1), (16, 2), (24, 2), (32, 2)])
def test_deposit_bit_exact(ctx, scheme, n, ss):
    box = 200.0
    xyz = synth.uniform_catalogue(3001, box, seed=n * 7 + ss)
    # edges: exactly 0, just below L, a node position
    xyz[:3] = [[0.0, 0.0, 0.0], [np.nextafter(box, 0), np.nextafter(box, 0), 0.0],
               [box / 2, box / n, box / (2 * n)]]
    w = synth.cap_mask(n, box, 70.0, 120.0)
    ctx.set_grid(n, box)
    ctx.set_mask(w)
    ctx.set_galaxies(xyz)
    ctx.deposit(scheme, ss)
    fine, nobs, nbar = ctx.get_deposit(True, True, ss)
    ref_grid = od.deposit(xyz, ss * n, box, scheme)
    assert np.array_equal(fine, ref_grid)
    ref_nobs, _ = oss.observed_counts(xyz, n, box, scheme, ss)
    assert rel_max(nobs, ref_nobs) < 1e-13
    assert nbar == pytest.approx(ow.mean_density(len(xyz), w), rel=1e-15)


def test_deposit_empty_catalogue(ctx):
    n = 16
    ctx.set_grid(n, 100.0)
    ctx.set_mask(np.full((n, n, n), 0.5))
    ctx.set_galaxies(np.zeros((0, 3)))
    ctx.deposit("tsc", 2)
    fine, nobs, nbar = ctx.get_deposit(True, True, 2)
    assert not fine.any() and not nobs.any() and nbar == 0.0


def test_deposit_order_independent(ctx):
    n, box = 32, 100.0
    xyz = synth.uniform_catalogue(20000, box, seed=3)
    # clustered: many galaxies in a few cells stress the integer atomics
    xyz[:5000] = 50.0 + 0.01 * (xyz[:5000] / box)
    ctx.set_grid(n, box)
    ctx.set_mask(np.ones((n, n, n)))
    ctx.set_galaxies(xyz)
    ctx.deposit("tsc", 2)
    g1, _, _ = ctx.get_deposit(True, False, 2)
    perm = np.random.Generator(np.random.PCG64(1)).permutation(len(xyz))
    ctx.set_galaxies(np.ascontiguousarray(xyz[perm]))
    ctx.deposit("tsc", 2)
    g2, _, _ = ctx.get_deposit(True, False, 2)
    assert np.array_equal(g1, g2)
    assert int(g1.sum()) == len(xyz) << 39


@pytest.mark.parametrize("scheme", ["cic", "tsc"])
def test_deposit_piled_on_one_point(ctx, scheme):
    """The degenerate catalogue of the contention measurement: 200 000
    galaxies at one position, every one of them adding to the same 8 or 27
    fine nodes.  Integer atomics make the grid exact whatever the order in
    which the adds land: equal to the oracle's, total N_gal 2^39."""
    n, box, ngal = 32, 100.0, 200_000
    p = 0.5 * box + 0.3 * box / (2 * n)
    xyz = np.full((ngal, 3), p)
    ctx.set_grid(n, box)
    ctx.set_mask(np.ones((n, n, n)))
    ctx.set_galaxies(xyz)
    ctx.deposit(scheme, 2)
    fine, _, _ = ctx.get_deposit(True, False, 2)
    assert np.array_equal(fine, od.deposit(xyz, 2 * n, box, scheme))
    assert int(fine.sum()) == ngal << 39
    assert np.count_nonzero(fine) == (8 if scheme == "cic" else 27)


def test_supersample_after_a_larger_grid(ctx):
    """One context reused from a larger to smaller grids: the fine-grid FFT
    tables follow the grid (a 48^3 fine grid after a 64^3 one once kept the
    64-point twiddles)."""
    box = 150.0
    for n in (32, 24, 16):
        xyz = synth.uniform_catalogue(4000, box, seed=100 + n)
        w = synth.cap_mask(n, box, 70.0, 120.0)
        ctx.set_grid(n, box)
        ctx.set_mask(w)
        ctx.set_galaxies(xyz)
        ctx.deposit("cic", 2)
        _, nobs, _ = ctx.get_deposit(False, True, 2)
        ref_nobs, _ = oss.observed_counts(xyz, n, box, "cic", 2)
        assert rel_max(nobs, ref_nobs) < 1e-13
