"""Pins of the oracle's signal-dependent noise formulation (eq:noisecov,
Sec. 3.4): the counter-based generator, the count estimators and the SD
Wiener system against a dense solve written from the definitions."""
import math
import os

import numpy as np
import pytest

import synth
from oracle import sdnoise as sd
from oracle import wiener as ow

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _kat():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append([int(x, 16) for x in line.split()])
    return rows


@pytest.mark.parametrize("row", _kat())
def test_philox_known_answers(row):
    out = sd.philox4x32_10(row[0:4], row[4:6])
    assert [int(x) for x in out] == row[6:10]


def test_philox_words_are_uniform():
    u = sd.keep_draws(1 << 20, 3, 12345).astype(np.float64) / 2.0 ** 32
    # mean 1/2, variance 1/12: five standard errors
    assert abs(u.mean() - 0.5) < 5 * math.sqrt(1 / 12 / u.size)
    assert abs(u.var() - 1 / 12) < 5 * math.sqrt(1 / 180 / u.size)
    assert not np.array_equal(sd.keep_draws(1000, 3, 12345), sd.keep_draws(1000, 4, 12345))
    assert not np.array_equal(sd.keep_draws(1000, 3, 12345), sd.keep_draws(1000, 3, 12346))


def _nodes_catalogue(n, box, nodes, per_node, seed=0):
    """Galaxies within a quarter cell of given nodes (nearest node known)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h = box / n
    pts = []
    for (i, j, k), c in zip(nodes, per_node):
        base = np.array([i, j, k], dtype=np.float64) * h
        pts.append(base + rng.uniform(-0.25 * h, 0.25 * h, size=(c, 3)))
    return np.mod(np.concatenate(pts), box)


def test_counts_and_mean_estimator():
    n, box = 8, 80.0
    nodes = [(0, 0, 0), (3, 4, 5), (7, 7, 7)]
    xyz = _nodes_catalogue(n, box, nodes, [2, 5, 1])
    c = sd.ngp_counts(xyz, n, box)
    assert c.sum() == 8 and c[0, 0, 0] == 2 and c[3, 4, 5] == 5 and c[7, 7, 7] == 1
    lam = sd.lambda_obs_mean(c)
    assert lam[3, 4, 5] == 6.0 and lam[1, 1, 1] == 1.0
    w = np.ones((n, n, n))
    w[3, 4, 5] = 0.0
    assert sd.ngp_counts(xyz, n, box, w)[3, 4, 5] == 0


def test_thinning_limits():
    n, box = 8, 80.0
    xyz = synth.uniform_catalogue(3000, box, seed=2)
    w = np.full((n, n, n), 0.4)
    # alpha = w: keep probability one, the full counts
    assert np.array_equal(sd.thinned_counts(xyz, n, box, w, 0.4, 9, 0), sd.ngp_counts(xyz, n, box))
    # and then the jackknife estimate is the mean estimator
    t = sd.thinned_counts(xyz, n, box, w, 0.4, 9, 0)
    assert np.allclose(sd.lambda_obs_jackknife(t, w, 0.4), sd.lambda_obs_mean(t), rtol=1e-15)
    with pytest.raises(ValueError):
        sd.thinned_counts(xyz, n, box, w, 0.41, 9, 0)
    assert sd.thinned_counts(xyz, n, box, w, 1e-12, 9, 0).sum() == 0


def test_thinning_is_binomial():
    n, box = 4, 40.0
    xyz = synth.uniform_catalogue(2000, box, seed=3)
    w = np.where(np.arange(n ** 3).reshape(n, n, n) % 2 == 0, 0.5, 0.8)
    alpha = 0.3
    full = sd.ngp_counts(xyz, n, box).astype(np.float64)
    p = alpha / w
    draws = np.array([sd.thinned_counts(xyz, n, box, w, alpha, 77, j) for j in range(300)],
                     dtype=np.float64)
    mean = draws.mean(axis=0)
    var = draws.var(axis=0)
    se = np.sqrt(full * p * (1 - p) / draws.shape[0])
    assert np.all(np.abs(mean - full * p) < 5 * se + 1e-12)
    # the binomial variance N p (1 - p), to within its sampling error (~8 %)
    assert np.allclose(var.sum(), (full * p * (1 - p)).sum(), rtol=0.05)
    # the sample index and the seed change the draws; the same ones reproduce
    assert np.array_equal(draws[5], sd.thinned_counts(xyz, n, box, w, alpha, 77, 5))
    assert not np.array_equal(draws[5], draws[6])


def _setup(n=6, box=60.0, seed=4):
    wl = synth.Workload("sd6", n, box, "cic", 1, 600, seed, "bbks", theta_deg=80.0, r0=40.0)
    ptab = wl.ptab()
    w = wl.mask()
    xyz = wl.catalogue(ptab, w).xyz
    from oracle import supersample as oss
    nobs, _ = oss.observed_counts(xyz, n, box, "cic", 1)
    nbar = ow.mean_density(len(xyz), w)
    return wl, ptab, w, xyz, nobs, nbar


def test_lsq_noise_gives_the_lsq_system():
    wl, ptab, w, xyz, nobs, nbar = _setup()
    base = ow.System(wl.n, wl.box, w, ptab, nbar)
    sds = sd.SDSystem(wl.n, wl.box, w, ptab, nbar, np.where(w > 0, nbar * w, 1.0))
    v = np.random.Generator(np.random.PCG64(1)).standard_normal(w.shape)
    assert np.allclose(sds.apply(v), base.apply(v), rtol=1e-14, atol=1e-14)
    assert np.allclose(sds.data_vector(nobs), ow.data_vector(nobs, w, nbar), rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("kind", ["mean", "jackknife"])
def test_sd_system_against_a_dense_solve(kind):
    """(S^-1 + R N^-1 R) s = R N^-1 delta^o with R = diag(w), N = diag(lambda^o /
    nbar^2) and delta^o = (n^o - nbar w) / nbar, all as dense matrices on the
    observed cells, against CG on the oracle's SD system."""
    wl, ptab, w, xyz, nobs, nbar = _setup()
    n = wl.n
    if kind == "mean":
        lam = sd.lambda_obs_mean(sd.ngp_counts(xyz, n, wl.box, w))
    else:
        alpha = 0.8 * float(w[w > 0].min())
        lam = sd.lambda_obs_jackknife(sd.thinned_counts(xyz, n, wl.box, w, alpha, 5, 2), w, alpha)
    sds = sd.SDSystem(n, wl.box, w, ptab, nbar, lam)
    b = sds.data_vector(nobs)
    x = ow.cg(sds, b, 1e-13, 5000)["x"]
    # dense S^-1: the Fourier diagonal lambda_table applied to each unit vector
    # through numpy's complex FFT (not the oracle's real transforms)
    m = n ** 3
    lam_k = ow.lambda_table(ptab, wl.box, n)
    mm = np.fft.fftfreq(n, 1.0 / n).astype(np.int64)
    m2 = (mm[:, None, None] ** 2 + mm[None, :, None] ** 2 + mm[None, None, :] ** 2)
    sinv = np.empty((m, m))
    for i in range(m):
        e = np.zeros(m)
        e[i] = 1.0
        sinv[:, i] = np.fft.ifftn(lam_k[m2] * np.fft.fftn(e.reshape(n, n, n))).real.ravel()
    wf = w.ravel()
    obs = wf > 0
    ninv = np.zeros(m)
    ninv[obs] = nbar * nbar / lam.ravel()[obs]
    delta_o = np.where(obs, (nobs.ravel() - nbar * wf) / nbar, 0.0)
    a = sinv + np.diag(wf * ninv * wf)
    rhs = wf * ninv * delta_o
    s = np.linalg.solve(a, rhs)
    assert np.allclose(x.ravel(), s, rtol=0, atol=1e-9 * np.abs(s).max())
