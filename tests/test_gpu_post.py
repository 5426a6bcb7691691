"""GPU parity of the post-solve functions against the oracle (through the C
ABI): redshift-distortion factor, Fourier-diagonal filters, moments, the
Sec. 4.1 measures and the inverse-weighting comparator."""
import numpy as np
import pytest

import synth
from oracle import post as op

from gpu_util import context, rel_max

pytestmark = pytest.mark.gpu

BETA, SIGMA = 0.24 ** 0.6, 500.0 / 73.0   # beta = Omega_m^0.6, 500 km/s / H0 in Mpc


@pytest.fixture(scope="module")
def ctx():
    c = context()
    yield c
    c.close()


def _setup(ctx, n, box, seed=1):
    w = synth.cap_mask(n, box, 70.0, 0.6 * box)
    ctx.set_grid(n, box)
    ctx.set_mask(w)
    return w


@pytest.mark.parametrize("n,box", [(32, 500.0), (24, 300.0), (128, 100.0)])
def test_rsd_factor(ctx, n, box):
    _setup(ctx, n, box)
    got = ctx.rsd_factor(BETA, SIGMA)
    want = op.rsd_factor_table(n, box, BETA, SIGMA)
    assert rel_max(got, want) < 1e-12


@pytest.mark.parametrize("n", [16, 24, 32, 48])
def test_filters(ctx, n):
    box = 200.0
    _setup(ctx, n, box)
    v = np.random.Generator(np.random.PCG64(n)).standard_normal((n, n, n))
    got = ctx.fourier_filter(v, "gauss", a=7.5)
    assert rel_max(got, op.fourier_filter(v, op.gauss_table(n, box, 7.5))) < 1e-12
    got = ctx.fourier_filter(v, "rsd_deconv", a=BETA, b=SIGMA, c=1.2)
    assert rel_max(got, op.fourier_filter(v, op.deconv_table(n, box, BETA, SIGMA, 1.2))) < 1e-12
    h = np.random.Generator(np.random.PCG64(5)).uniform(0.5, 1.5, 3 * (n // 2) ** 2 + 1)
    got = ctx.fourier_filter(v, "table", table=h)
    assert rel_max(got, op.fourier_filter(v, h)) < 1e-12


def test_filter_rejects_bad_input(ctx):
    import paper_0906_3978_amd as wf
    _setup(ctx, 16, 100.0)
    v = np.zeros((16, 16, 16))
    with pytest.raises(wf.WienerError):
        ctx.fourier_filter(v, "table", table=np.zeros(10))
    h = np.ones(3 * 64 + 1)
    h[5] = np.inf
    with pytest.raises(wf.WienerError):
        ctx.fourier_filter(v, "table", table=h)


@pytest.mark.parametrize("masked", [False, True])
def test_moments_and_measures(ctx, masked):
    n, box = 32, 300.0
    w = _setup(ctx, n, box)
    rng = np.random.Generator(np.random.PCG64(9))
    a = rng.lognormal(0.0, 0.6, (n, n, n)) - 1.0
    b = a + 0.1 * rng.standard_normal((n, n, n))
    got = ctx.field_moments(a, masked=masked)
    want = op.moments(a, w if masked else None)
    assert got[0] == want[0]
    assert np.allclose(got[1:], want[1:], rtol=1e-11, atol=1e-14)
    got = ctx.compare_fields(b, a, masked=masked)
    want = op.compare(b, a, w if masked else None)
    assert np.allclose(got[:2], want[:2], rtol=1e-11)
    if np.isnan(want[2]):
        assert np.isnan(got[2])
    else:
        assert got[2] == pytest.approx(want[2], rel=1e-10)


@pytest.mark.parametrize("scheme,ss", [("ngp", 1), ("cic", 1), ("cic", 2), ("tsc", 2)])
def test_inverse_weighting(ctx, scheme, ss):
    n, box = 24, 240.0
    wl = synth.Workload("iw24", n, box, scheme, ss, 20000, 77, "bbks")
    ptab = wl.ptab()
    w = wl.mask()
    xyz = wl.catalogue(ptab, w).xyz
    ctx.set_grid(n, box)
    ctx.set_mask(w)
    ctx.set_galaxies(xyz)
    got = ctx.inverse_weighting(scheme, ss)
    want = op.inverse_weighting(xyz, n, box, w, scheme, ss)
    assert rel_max(got + 1.0, want + 1.0) < 1e-12


def test_redshift_space_prior_and_deconvolution(ctx):
    """Sec. 3.3.3: the prior in redshift space is <KD>_mu P; the solve with it,
    then eq:DEC with a constant bias, against the oracle's."""
    from oracle import wiener as ow
    wl = synth.Workload("rsd32", 32, 300.0, "cic", 2, 20000, 515, "bbks")
    ptab = wl.ptab()
    w = wl.mask()
    xyz = wl.catalogue(ptab, w).xyz
    ctx.set_grid(wl.n, wl.box)
    ctx.set_mask(w)
    ps = ptab * ctx.rsd_factor(BETA, SIGMA)
    ctx.set_power(ps)
    ctx.set_galaxies(xyz)
    ctx.deposit("cic", 2)
    x, info = ctx.solve(precision="fp64", precond="prior", tol=1e-12, max_iter=20000)
    ps_ref = ptab * op.rsd_factor_table(wl.n, wl.box, BETA, SIGMA)
    ref = ow.reconstruct(xyz, wl.n, wl.box, w, ps_ref, "cic", 2, 1e-12, 20000)
    assert rel_max(x, ref["x"]) < 1e-9
    dec = ctx.fourier_filter(x, "rsd_deconv", a=BETA, b=SIGMA, c=1.3)
    want = op.fourier_filter(ref["x"], op.deconv_table(wl.n, wl.box, BETA, SIGMA, 1.3))
    assert rel_max(dec, want) < 1e-9
