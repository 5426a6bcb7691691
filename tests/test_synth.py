"""Checks of the synthetic input generators (Sec. 3.2.2 observation law)."""
import numpy as np
from scipy import stats

import synth


def test_poisson_binomial_equals_thinned_poisson():
    """eq:poisbin: binomial thinning of Poisson(lambda) with acceptance w is
    Poisson(w lambda)."""
    rng = np.random.Generator(np.random.PCG64(1))
    lam, w = 3.7, 0.35
    n = 200_000
    a = synth.poisson_binomial_two_stage(np.full(n, lam), np.full(n, w), rng)
    b = synth.poisson_direct(np.full(n, lam), np.full(n, w), rng)
    kmax = 8
    ha = np.bincount(np.minimum(a, kmax), minlength=kmax + 1)
    hb = np.bincount(np.minimum(b, kmax), minlength=kmax + 1)
    chi2, p, _, _ = stats.chi2_contingency(np.vstack([ha, hb]))
    assert p > 0.01
    assert abs(a.mean() - w * lam) < 5 * np.sqrt(w * lam / n)


def test_lognormal_mean_and_variance():
    n, box = 32, 256.0
    ptab = synth.p_by_m2(synth.power_law_normalised(32, 256.0, 0.5), n, box)
    assert abs(synth.cell_variance(ptab, n, box) - 0.5) < 1e-12
    g = synth.gaussian_field(ptab, n, box, seed=3)
    assert abs(g.mean()) < 1e-12
    assert 0.3 < g.var() < 0.7
    opd, s2 = synth.lognormal_density(ptab, n, box, seed=3)
    assert np.all(opd > 0)
    assert abs(opd.mean() - 1.0) < 0.1


def test_cap_mask_properties():
    w = synth.cap_mask(32, 256.0, 60.0, 150.0)
    assert w.max() <= 1.0 and w.min() >= 0.0
    assert w[16, 16, 16] == 1.0
    assert w[16, 16, 0] == 0.0        # straight below the observer: outside the cap
    assert w[16, 16, 31] > 0.0        # along the axis: inside
    frac = (w > 0).mean()
    assert 0.05 < frac < 0.5


def test_catalogue_in_box_and_count():
    wl = synth.workload("pl32")
    cat = wl.catalogue()
    assert cat.xyz.shape[1] == 3
    assert np.all(cat.xyz >= 0) and np.all(cat.xyz < wl.box)
    assert abs(len(cat.xyz) - wl.n_target) < 6 * np.sqrt(wl.n_target)
    assert cat.counts.sum() == len(cat.xyz)


def test_bbks_positive_and_sigma8():
    k = np.logspace(-3, 1, 50)
    p = synth.bbks_power(k)
    assert np.all(p > 0)
    assert synth.m2_table_len(512) == 196609
