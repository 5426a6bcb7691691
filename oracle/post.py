"""After the solve (oracle; test infrastructure only): the angle-averaged
redshift-distortion factor and the deconvolution of Sec. 3.3.2-3.3.3, the
Gaussian smoothing, the inverse-weighting comparator and the quality measures
of Sec. 4.

Readings taken here:

* the angle average of Sec. 3.3.3 runs over mu in [0, 1] (the integrand is
  even in mu), sigma is a length (the paper's 500 km/s / H0);
* eq:DEC with a constant bias b: the filter 1 / (b sqrt(<K D>_mu(k)));
* eq:GAUSS is read with the minus sign, exp(-|r|^2 / (2 r_S^2)), normalised
  to unit integral, i.e. exp(-k^2 r_S^2 / 2) in Fourier space;
* inverse weighting: each galaxy carries 1/w of the target node nearest to it
  (the same fixed-point rule as the NGP deposit on the target grid), is
  deposited with the chosen kernel on the supersampled grid and low-passed like
  n^o; delta_IW = n_IW / nbar - 1 with nbar of eq:nmean;
* r, D_Euc and D_KL as printed in Sec. 4.1, over every cell of the field (or
  the cells with w > 0); D_KL needs 1 + delta > 0 everywhere.
"""
from __future__ import annotations

import math

import numpy as np

from .deposit import F_BITS, HALF, fixed_point, galaxy_stencils, scheme_unit
from .supersample import lowpass_decimate
from .wiener import m2_half_grid


def _gauss_legendre(f, lo, hi, panel=0.5, order=20):
    """int_lo^hi f by composite Gauss-Legendre quadrature: panels of length
    at most `panel`, `order` nodes each.  For an integrand analytic within
    distance 1 of the real interval (the case below) a 20-node rule on
    half-unit panels is exact to rounding (Bernstein-ellipse bound
    ~8^-40)."""
    x, w = np.polynomial.legendre.leggauss(order)
    m = max(1, int(math.ceil((hi - lo) / panel)))
    edges = np.linspace(lo, hi, m + 1)
    half = 0.5 * (edges[1:] - edges[:-1])
    mid = 0.5 * (edges[1:] + edges[:-1])
    t = mid[:, None] + half[:, None] * x[None, :]
    return float(np.sum(half[:, None] * w[None, :] * f(t)))


def rsd_factor(k, beta, sigma):
    """<K D>_mu(k): int_0^1 (1 + beta mu^2)^2 / (1 + k^2 sigma^2 mu^2 / 2) dmu
    (Kaiser factor times the Lorentzian damping, angle averaged).  For
    a = k^2 sigma^2 / 2 > 1 the same integral is taken in t = sqrt(a) mu,
    (1 / sqrt(a)) int_0^sqrt(a) (1 + beta t^2 / a)^2 / (1 + t^2) dt, where the
    Lorentzian has unit width.  Either way the integrand's poles lie at
    distance >= 1 from the real interval, and the composite Gauss-Legendre
    rule above reaches rounding level."""
    def one(kk):
        a = 0.5 * kk * kk * sigma * sigma
        if a <= 1.0:
            return _gauss_legendre(lambda mu: (1 + beta * mu * mu) ** 2 / (1 + a * mu * mu),
                                   0.0, 1.0)
        ra = math.sqrt(a)
        return _gauss_legendre(lambda t: (1 + beta * t * t / a) ** 2 / (1 + t * t), 0.0, ra) / ra
    return np.array([one(float(kk)) for kk in np.atleast_1d(k)])


def rsd_factor_table(n, box, beta, sigma, length=None):
    """<K D>_mu at k = (2 pi / L) sqrt(j), j < length."""
    length = length or 3 * (n // 2) ** 2 + 1
    k = (2.0 * math.pi / box) * np.sqrt(np.arange(length, dtype=np.float64))
    return rsd_factor(k, beta, sigma)


def gauss_table(n, box, r_s):
    """exp(-k^2 r_S^2 / 2) on the |m|^2 lattice (eq:GAUSS)."""
    j = np.arange(3 * (n // 2) ** 2 + 1, dtype=np.float64)
    k2 = (2.0 * math.pi / box) ** 2 * j
    return np.exp(-0.5 * k2 * r_s * r_s)


def deconv_table(n, box, beta, sigma, bias):
    """1 / (b sqrt(<K D>_mu)) on the |m|^2 lattice (eq:DEC)."""
    return 1.0 / (bias * np.sqrt(rsd_factor_table(n, box, beta, sigma)))


def fourier_filter(v, h_by_m2):
    """F^-1 diag(h(|m|^2)) F v on a periodic n^3 grid."""
    n = v.shape[0]
    return np.fft.irfftn(h_by_m2[m2_half_grid(n)] * np.fft.rfftn(v), s=v.shape, axes=(0, 1, 2))


def moments(v, w=None):
    """(count, mean, variance, skewness, excess kurtosis), population moments."""
    x = np.asarray(v, dtype=np.float64).ravel()
    if w is not None:
        x = x[np.asarray(w).ravel() > 0]
    n = x.size
    mu = x.mean()
    d = x - mu
    var = float(np.mean(d * d))
    return (float(n), float(mu), var, float(np.mean(d ** 3)) / var ** 1.5,
            float(np.mean(d ** 4)) / var ** 2 - 3.0)


def compare(rec, tru, w=None):
    """Sec. 4.1: correlation coefficient r, Euclidean distance D_Euc and
    Kullback-Leibler distance D_KL(1 + rec, 1 + tru)."""
    r = np.asarray(rec, dtype=np.float64).ravel()
    t = np.asarray(tru, dtype=np.float64).ravel()
    if w is not None:
        keep = np.asarray(w).ravel() > 0
        r, t = r[keep], t[keep]
    n = r.size
    corr = float(np.sum(t * r) / (math.sqrt(float(np.sum(t * t))) * math.sqrt(float(np.sum(r * r)))))
    deuc = math.sqrt(float(np.sum((r - t) ** 2)) / n)
    if np.all(1 + r > 0) and np.all(1 + t > 0):
        dkl = float(np.sum((1 + r) * np.log((1 + r) / (1 + t)))) / n
    else:
        dkl = float("nan")
    return corr, deuc, dkl


def nearest_node(xyz, n, box):
    """Flat index of the target node nearest to each galaxy (the NGP rule)."""
    U = fixed_point(xyz, n, box)
    node = ((U + HALF) >> F_BITS) % n
    return (node[:, 0] * n + node[:, 1]) * n + node[:, 2]


def inverse_weighting(xyz, n, box, w, scheme, supersample):
    """delta_IW on the n^3 grid."""
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    wf = np.asarray(w, dtype=np.float64).ravel()
    wg = wf[nearest_node(xyz, n, box)]
    if np.any(wg <= 0):
        raise ValueError("a galaxy lies on a node with w = 0")
    n_d = supersample * n
    grid = np.zeros(n_d ** 3, dtype=np.float64)
    idx, wt = galaxy_stencils(xyz, n_d, box, scheme)
    per = wt.size // xyz.shape[0]
    np.add.at(grid, idx, wt.astype(np.float64) * scheme_unit(scheme) * np.repeat(1.0 / wg, per))
    g = grid.reshape(n_d, n_d, n_d)
    n_iw = g if supersample == 1 else lowpass_decimate(g, n)
    nbar = xyz.shape[0] / float(wf.sum())
    return n_iw / nbar - 1.0
