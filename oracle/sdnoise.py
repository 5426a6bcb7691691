"""Signal-dependent noise formulation of the Wiener filter (oracle; test
infrastructure only): eq:noisecov with the estimators of Sec. 3.4 for the
expected observed count lambda^o = w lambda.

The system keeps the signal-space form of eq:WF with R = diag(w), the data
delta^o = (n^o - nbar w) / nbar and N = diag(lambda^o / nbar^2) per cell:

    (S^-1 + diag(nbar^2 w^2 / lambda^o)) s = nbar w (n^o - nbar w) / lambda^o

on cells with w > 0 (cells with w = 0 carry neither data nor noise term, as
in the LSQ form).  With g = nbar w / lambda^o this is A_g = F^-1 Lambda F +
diag(nbar w g), b_g = g (n^o - nbar w); lambda^o = nbar w gives g = 1, the
LSQ system.

Readings taken here:

* the counts N^o_c of the estimators are the galaxies whose nearest target
  node is the cell (the NGP rule on the target grid; the paper neglects the
  gridding correlation in eq:noisecov too);
* flat-prior mean estimator: lambda^o_mean = N^o_c + 1;
* jackknife: each galaxy is kept with probability alpha / w of its node
  (so N' ~ Bin(N^o_c, alpha / w)), and the kept counts give
  lambda^o_JK = w (N' + 1) / alpha -- the flat-prior mean of the thinned
  Poisson rate alpha lambda, scaled back by 1 / alpha; without the + 1 a cell
  with N' = 0 would have zero noise and an infinite weight;
* alpha must not exceed w on any observed node (the keep probability is at
  most 1);
* the random draws come from Philox4x32-10 (Salmon et al. 2011, "Parallel
  random numbers: as easy as 1, 2, 3") with counter (galaxy index low word,
  galaxy index high word, sample index, 0) and key (seed low word, seed high
  word); galaxy g is kept in sample j when the first output word u satisfies
  u < (alpha / w) 2^32, compared in FP64 (both sides exact);
* the data vector n^o is the full observed sample in every jackknife sample;
  the samples differ only in their noise estimate, and the reconstruction is
  their mean.
"""
from __future__ import annotations

import numpy as np

from .post import nearest_node
from .wiener import System

PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
MASK32 = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds.  ctr: four uint32 arrays (broadcastable),
    key: two uint32 arrays.  Returns the four output words (uint64 arrays
    holding 32-bit values)."""
    c = [np.asarray(x, dtype=np.uint64) & MASK32 for x in ctr]
    k0 = np.asarray(key[0], dtype=np.uint64) & MASK32
    k1 = np.asarray(key[1], dtype=np.uint64) & MASK32
    for rnd in range(10):
        if rnd:
            k0 = (k0 + PHILOX_W0) & MASK32
            k1 = (k1 + PHILOX_W1) & MASK32
        p0 = np.uint64(PHILOX_M0) * c[0]      # < 2^64: exact in uint64
        p1 = np.uint64(PHILOX_M1) * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return c


def ngp_counts(xyz, n, box, w=None):
    """N^o_c: galaxies per nearest target node (only nodes with w > 0 if w is
    given)."""
    node = nearest_node(xyz, n, box)
    cnt = np.bincount(node, minlength=n ** 3)
    if w is not None:
        cnt = np.where(np.asarray(w).ravel() > 0, cnt, 0)
    return cnt.reshape(n, n, n)


def keep_draws(n_gal, sample, seed):
    """First Philox word for every galaxy of one jackknife sample."""
    g = np.arange(n_gal, dtype=np.uint64)
    key = (np.uint64(seed & MASK32), np.uint64((seed >> 32) & MASK32))
    return philox4x32_10((g & MASK32, g >> np.uint64(32), np.uint64(sample), np.uint64(0)), key)[0]


def thinned_counts(xyz, n, box, w, alpha, seed, sample):
    """N'_c of eq:selfunc for one jackknife sample: binomial thinning with
    keep probability alpha / w(node)."""
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    wf = np.asarray(w, dtype=np.float64).ravel()
    node = nearest_node(xyz, n, box)
    wn = wf[node]
    obs = wn > 0
    if np.any(alpha > wn[obs]):
        raise ValueError("alpha exceeds w on an observed node")
    p = np.zeros_like(wn)
    p[obs] = alpha / wn[obs]
    u = keep_draws(len(xyz), sample, seed).astype(np.float64)
    keep = obs & (u < p * 4294967296.0)
    return np.bincount(node[keep], minlength=n ** 3).reshape(n, n, n)


def lambda_obs_mean(counts):
    """Flat-prior mean estimator of Sec. 3.4.1: w lambda_mean = N^o_c + 1."""
    return np.asarray(counts, dtype=np.float64) + 1.0


def lambda_obs_jackknife(thinned, w, alpha):
    """w (N' + 1) / alpha (the jackknife-like scheme of Sec. 3.4.2, read with
    the flat-prior + 1)."""
    return np.asarray(w, dtype=np.float64) * (np.asarray(thinned, dtype=np.float64) + 1.0) / alpha


class SDSystem(System):
    """A_g s = b_g with g = nbar w / lambda^o on w > 0 (module docstring)."""

    def __init__(self, n, box, w, p_by_m2, nbar, lambda_obs, workers=None):
        super().__init__(n, box, w, p_by_m2, nbar, workers)
        lo = np.asarray(lambda_obs, dtype=np.float64)
        obs = self.w > 0
        if np.any(lo[obs] <= 0):
            raise ValueError("lambda^o must be > 0 on observed cells")
        self.g = np.zeros_like(self.w)
        self.g[obs] = self.nbar * self.w[obs] / lo[obs]
        # diag(nbar^2 w^2 / lambda^o) = nbar w g
        self.nw = self.nbar * self.w * self.g

    def data_vector(self, n_obs):
        """nbar w (n^o - nbar w) / lambda^o = g (n^o - nbar w) on w > 0."""
        return np.where(self.w > 0, self.g * (np.asarray(n_obs) - self.nbar * self.w), 0.0)
