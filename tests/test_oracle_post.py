"""Pins of the oracle's post-solve functions: the redshift-distortion factor and
deconvolution (Sec. 3.3.3, eq:DEC), Gaussian smoothing (eq:GAUSS), the quality
measures of Sec. 4.1 and the inverse-weighting comparator (Sec. 4)."""
import math

import numpy as np
import pytest

from oracle import post as op
from oracle import supersample as oss
import synth


@pytest.mark.parametrize("beta", [0.0, 0.42, 1.3])
def test_rsd_factor_without_damping_is_the_kaiser_average(beta):
    # int_0^1 (1 + beta mu^2)^2 dmu = 1 + 2 beta / 3 + beta^2 / 5
    got = op.rsd_factor(np.array([0.0, 0.3, 2.0]), beta, 0.0)
    assert np.allclose(got, 1 + 2 * beta / 3 + beta * beta / 5, rtol=1e-13, atol=0)


@pytest.mark.parametrize("k", [0.01, 0.2, 1.0, 5.0])
def test_rsd_factor_without_kaiser_is_the_lorentzian_average(k):
    sigma = 6.85
    a = 0.5 * k * k * sigma * sigma
    want = math.atan(math.sqrt(a)) / math.sqrt(a)
    assert op.rsd_factor(np.array([k]), 0.0, sigma)[0] == pytest.approx(want, rel=1e-12)


@pytest.mark.parametrize("k,beta", [(0.05, 0.42), (0.7, 0.42), (4.0, 0.9)])
def test_rsd_factor_against_a_midpoint_sum(k, beta):
    sigma = 6.85
    mu = (np.arange(2_000_000) + 0.5) / 2_000_000
    brute = float(np.mean((1 + beta * mu * mu) ** 2 / (1 + 0.5 * k * k * sigma * sigma * mu * mu)))
    assert op.rsd_factor(np.array([k]), beta, sigma)[0] == pytest.approx(brute, rel=1e-9)


def _cos_mode(n, m):
    x = np.arange(n)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    return np.cos(2 * np.pi * (m[0] * X + m[1] * Y + m[2] * Z) / n)


def test_gauss_filter_on_a_fourier_mode():
    n, box, r_s = 16, 100.0, 7.0
    m = (2, -3, 1)
    v = _cos_mode(n, m)
    k2 = (2 * math.pi / box) ** 2 * sum(c * c for c in m)
    got = op.fourier_filter(v, op.gauss_table(n, box, r_s))
    assert np.allclose(got, math.exp(-0.5 * k2 * r_s * r_s) * v, atol=1e-13)


def test_gauss_filter_keeps_the_mean_and_smooths_a_spike():
    n, box = 32, 100.0
    v = np.zeros((n, n, n))
    v[5, 6, 7] = 1.0
    out = op.fourier_filter(v, op.gauss_table(n, box, 8.0))
    assert out.sum() == pytest.approx(1.0, rel=1e-12)
    # a Gaussian of width 8 Mpc sampled at H = 3.125 Mpc: the peak stays where it was
    assert np.unravel_index(np.argmax(out), out.shape) == (5, 6, 7)


def _rsd_closed_form(k, beta, sigma):
    """<K D>_mu by polynomial division of the integrand: with a = k^2 sigma^2
    / 2, (1 + beta mu^2)^2 = (1 + a mu^2)(A mu^2 + B) + C with A = beta^2 / a,
    B = (2 beta - A) / a, C = 1 - B, so the mu-average over [0, 1] is
    A / 3 + B + C atan(sqrt(a)) / sqrt(a)."""
    a = 0.5 * k * k * sigma * sigma
    A = beta * beta / a
    B = (2 * beta - A) / a
    C = 1.0 - B
    return A / 3 + B + C * math.atan(math.sqrt(a)) / math.sqrt(a)


@pytest.mark.parametrize("k", [0.08, 0.5, 3.0])
def test_rsd_factor_closed_form(k):
    beta, sigma = 0.42, 6.85
    assert op.rsd_factor(np.array([k]), beta, sigma)[0] == pytest.approx(
        _rsd_closed_form(k, beta, sigma), rel=1e-12)


@pytest.mark.parametrize("n,box", [(8, 100.0), (24, 300.0), (32, 500.0), (128, 100.0)])
def test_rsd_factor_table_quadrature_is_quiet(n, box):
    """The factor tables of the GPU tests' grids, with every warning an
    error (the quadrature must reach its accuracy without complaint)."""
    import warnings
    with warnings.catch_warnings():
        warnings.simplefilter("error")
        op.rsd_factor_table(n, box, 0.24 ** 0.6, 500.0 / 73.0)


@pytest.mark.parametrize("m", [(3, 1, 2), (0, -5, 4), (7, 7, 0)])
def test_deconvolution_on_a_fourier_mode(m):
    """A single mode through the eq:DEC filter with beta, sigma != 0 comes
    out scaled by 1 / (b sqrt(<K D>_mu(k))) at k = (2 pi / L) |m|: pins the
    k lattice of the tables and the factor away from every limit."""
    n, box, beta, sigma, bias = 16, 120.0, 0.42, 6.85, 1.3
    v = _cos_mode(n, m)
    k = 2 * math.pi / box * math.sqrt(sum(c * c for c in m))
    h = 1.0 / (bias * math.sqrt(_rsd_closed_form(k, beta, sigma)))
    got = op.fourier_filter(v, op.deconv_table(n, box, beta, sigma, bias))
    assert np.allclose(got, h * v, rtol=0, atol=1e-13)
    # and the redshift-space prior factor of the same mode, straight from the table
    tab = op.rsd_factor_table(n, box, beta, sigma)
    assert tab[sum(c * c for c in m)] == pytest.approx(_rsd_closed_form(k, beta, sigma), rel=1e-12)


def test_deconvolution_reduces_to_the_bias():
    n, box = 16, 100.0
    v = np.random.Generator(np.random.PCG64(1)).standard_normal((n, n, n))
    out = op.fourier_filter(v, op.deconv_table(n, box, 0.0, 0.0, 1.7))
    assert np.allclose(out, v / 1.7, atol=1e-13)


def test_filters_compose():
    n, box = 16, 80.0
    v = np.random.Generator(np.random.PCG64(2)).standard_normal((n, n, n))
    h1 = op.gauss_table(n, box, 5.0)
    h2 = op.deconv_table(n, box, 0.42, 6.85, 1.0)
    a = op.fourier_filter(op.fourier_filter(v, h1), h2)
    b = op.fourier_filter(v, h1 * h2)
    assert np.allclose(a, b, atol=1e-12)


@pytest.mark.parametrize("p", [0.1, 0.5, 0.73])
def test_moments_of_a_two_valued_field(p):
    n = 20
    v = np.zeros(n ** 3)
    k = int(round(p * v.size))
    v[:k] = 1.0
    p = k / v.size
    cnt, mean, var, skew, kurt = op.moments(v.reshape(n, n, n))
    q = 1 - p
    assert cnt == n ** 3
    assert mean == pytest.approx(p, rel=1e-13)
    assert var == pytest.approx(p * q, rel=1e-12)
    assert skew == pytest.approx((q - p) / math.sqrt(p * q), rel=1e-10, abs=1e-12)
    assert kurt == pytest.approx((1 - 6 * p * q) / (p * q), rel=1e-10, abs=1e-12)


def test_moments_masked_counts_observed_cells_only():
    v = np.arange(27, dtype=float).reshape(3, 3, 3)
    w = np.zeros((3, 3, 3))
    w[0, 0, :2] = 0.5  # cells 0 and 1
    cnt, mean, var, _, _ = op.moments(v, w)
    assert (cnt, mean, var) == (2.0, 0.5, 0.25)


def test_compare_measures():
    rng = np.random.Generator(np.random.PCG64(3))
    x = rng.uniform(-0.5, 2.0, size=(8, 8, 8))
    r, d, kl = op.compare(x, x)
    assert (r, d, kl) == (pytest.approx(1.0, rel=1e-14), 0.0, 0.0)
    assert op.compare(2 * x, x)[0] == pytest.approx(1.0, rel=1e-14)
    assert op.compare(-x, x)[0] == pytest.approx(-1.0, rel=1e-14)
    assert op.compare(x + 0.25, x)[1] == pytest.approx(0.25, rel=1e-12)
    # two cells, by hand
    rec = np.array([0.0, 1.0])
    tru = np.array([1.0, 0.0])
    r, d, kl = op.compare(rec, tru)
    assert r == 0.0 and d == pytest.approx(1.0) and kl == pytest.approx(0.5 * (-math.log(2) + 2 * math.log(2)))
    assert math.isnan(op.compare(np.array([-1.5, 0.0]), tru)[2])


@pytest.mark.parametrize("scheme,ss", [("ngp", 1), ("cic", 2), ("tsc", 2)])
def test_inverse_weighting_with_uniform_completeness_is_the_overdensity(scheme, ss):
    n, box = 16, 120.0
    xyz = synth.uniform_catalogue(5000, box, seed=7)
    nobs, _ = oss.observed_counts(xyz, n, box, scheme, ss)
    for c in (1.0, 0.25):
        w = np.full((n, n, n), c)
        got = op.inverse_weighting(xyz, n, box, w, scheme, ss)
        # 1/w on every galaxy and nbar = N / (c M) cancel
        want = nobs / (len(xyz) / n ** 3) - 1.0
        assert np.allclose(got, want, atol=1e-11)


def test_inverse_weighting_single_galaxy():
    n, box = 8, 80.0
    w = np.full((n, n, n), 1.0)
    w[3, 4, 5] = 0.5
    xyz = np.array([[3 * 10.0 + 1.0, 4 * 10.0 - 2.0, 5 * 10.0 + 4.9]])  # nearest node (3, 4, 5)
    got = op.inverse_weighting(xyz, n, box, w, "ngp", 1)
    nbar = 1 / w.sum()
    assert got[3, 4, 5] == pytest.approx(2.0 / nbar - 1.0, rel=1e-14)
    assert np.all(np.delete(got.ravel(), (3 * n + 4) * n + 5) == -1.0)
    w[3, 4, 5] = 0.0
    with pytest.raises(ValueError):
        op.inverse_weighting(xyz, n, box, w, "ngp", 1)
