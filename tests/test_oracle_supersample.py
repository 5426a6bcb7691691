"""Pins of the oracle's supersampling low-pass (Sec. 3.1.2) and of the FFT it
uses."""
import numpy as np
import pytest

from oracle import deposit as od
from oracle import supersample as oss
import synth


def _naive_dft3(x):
    n0, n1, n2 = x.shape
    out = np.zeros(x.shape, dtype=np.complex128)
    for k0 in range(n0):
        for k1 in range(n1):
            for k2 in range(n2):
                acc = 0j
                for a in range(n0):
                    for b in range(n1):
                        for c in range(n2):
                            ang = -2 * np.pi * (k0 * a / n0 + k1 * b / n1 + k2 * c / n2)
                            acc += x[a, b, c] * complex(np.cos(ang), np.sin(ang))
                out[k0, k1, k2] = acc
    return out


@pytest.mark.parametrize("n", [4, 6])
def test_numpy_fft_matches_naive_dft(n):
    x = np.random.Generator(np.random.PCG64(n)).standard_normal((n, n, n))
    ref = _naive_dft3(x)
    half = np.fft.rfftn(x)
    assert np.allclose(half, ref[:, :, :n // 2 + 1], rtol=0, atol=1e-11)
    assert np.allclose(np.fft.irfftn(half, s=x.shape, axes=(0, 1, 2)), x, rtol=0, atol=1e-13)


def test_parseval():
    x = np.random.Generator(np.random.PCG64(1)).standard_normal((12, 12, 12))
    X = np.fft.fftn(x)
    assert np.isclose((np.abs(X) ** 2).sum() / x.size, (x * x).sum(), rtol=1e-13)


@pytest.mark.parametrize("scheme", ["ngp", "cic", "tsc"])
def test_mass_preserved(scheme):
    xyz = synth.uniform_catalogue(3000, 200.0, seed=21)
    n_obs, grid = oss.observed_counts(xyz, 16, 200.0, scheme, 2)
    assert n_obs.shape == (16, 16, 16)
    assert abs(n_obs.sum() - 3000) <= 1e-12 * 3000


def _c1d(n, fine_hat):
    """(1/n) sum_{|m|<n/2} fine_hat(m) exp(2 pi i m j / n) for j = 0..n-1, by
    an explicit loop."""
    out = np.zeros(n)
    for j in range(n):
        acc = 0j
        for m in range(-(n // 2) + 1, n // 2):
            acc += fine_hat(m) * np.exp(2j * np.pi * m * j / n)
        out[j] = acc.real / n
    return out


def test_single_galaxy_tsc_closed_form():
    n, box = 8, 80.0
    # galaxy exactly on fine node 0: per-axis weights (1/8, 3/4, 1/8) on
    # nodes (-1, 0, +1); fine spectrum 3/4 + cos(pi m / n)/4.
    xyz = np.zeros((1, 3))
    n_obs, _ = oss.observed_counts(xyz, n, box, "tsc", 2)
    c = _c1d(n, lambda m: 0.75 + 0.25 * np.cos(np.pi * m / n))
    ref = c[:, None, None] * c[None, :, None] * c[None, None, :]
    assert np.allclose(n_obs, ref, rtol=0, atol=1e-14)


def test_single_galaxy_ngp_dirichlet():
    n, box = 10, 50.0
    xyz = np.array([[0.0, 0.0, 0.0]])
    n_obs, _ = oss.observed_counts(xyz, n, box, "ngp", 2)
    c = _c1d(n, lambda m: 1.0)
    ref = c[:, None, None] * c[None, :, None] * c[None, None, :]
    assert np.allclose(n_obs, ref, rtol=0, atol=1e-14)


def test_uniform_fine_field_is_uniform():
    # mass-conserving: each coarse cell holds the 8 fine cells it covers
    g = np.full((16, 16, 16), 3.25)
    out = oss.lowpass_decimate(g, 8)
    assert np.allclose(out, 8 * 3.25, rtol=0, atol=1e-13)


def test_idempotent_on_band_limited_field():
    n = 12
    rng = np.random.Generator(np.random.PCG64(4))
    f = rng.standard_normal((n, n, n))
    fk = np.fft.rfftn(f)
    h = n // 2
    fk[h, :, :] = 0
    fk[:, h, :] = 0
    fk[:, :, h] = 0
    f = np.fft.irfftn(fk, s=(n, n, n), axes=(0, 1, 2))
    # embed in the 2n spectrum (zero padding); the fine field then carries
    # 1/8 of each coarse cell's mass per fine cell, and decimation returns f
    big = np.zeros((2 * n, 2 * n, n + 1), dtype=np.complex128)
    keep_c = np.r_[0:h, n - h + 1:n]
    keep_f = np.r_[0:h, 2 * n - h + 1:2 * n]
    big[np.ix_(keep_f, keep_f, np.arange(h))] = fk[np.ix_(keep_c, keep_c, np.arange(h))]
    fine = np.fft.irfftn(big, s=(2 * n,) * 3, axes=(0, 1, 2))
    back = oss.lowpass_decimate(fine, n)
    assert np.allclose(back, f, rtol=0, atol=1e-13 * np.abs(f).max())


@pytest.mark.parametrize("scheme", ["ngp", "cic", "tsc"])
def test_direct_summation_matches_fft_route(scheme):
    n, box = 8, 64.0
    xyz = synth.uniform_catalogue(300, box, seed=31)
    n_obs, _ = oss.observed_counts(xyz, n, box, scheme, 2)
    rng = np.random.Generator(np.random.PCG64(5))
    cells = rng.integers(0, n, size=(12, 3))
    got = oss.observed_counts_at(xyz, n, box, scheme, cells)
    ref = n_obs[cells[:, 0], cells[:, 1], cells[:, 2]]
    assert np.allclose(got, ref, rtol=0, atol=1e-11)


def test_supersample_one_is_plain_deposit():
    xyz = synth.uniform_catalogue(500, 64.0, seed=2)
    n_obs, grid = oss.observed_counts(xyz, 8, 64.0, "cic", 1)
    assert np.array_equal(grid, od.deposit(xyz, 8, 64.0, "cic"))
    assert np.allclose(n_obs, grid * 2.0 ** -39, rtol=0, atol=0)


def test_threaded_fft_route_is_the_same_lowpass():
    """The optional multi-threaded FFT (scipy) gives the numpy route's field to
    rounding: the same transform, only the library differs."""
    rng = np.random.Generator(np.random.PCG64(5))
    g = rng.standard_normal((24, 24, 24))
    a = oss.lowpass_decimate(g, 12)
    b = oss.lowpass_decimate(g, 12, workers=4)
    assert np.abs(a - b).max() <= 1e-14 * np.abs(a).max()
