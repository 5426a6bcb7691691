"""Supersampling: ideal low-pass of the 2x deposit, resampled at the target
grid (oracle; test infrastructure only).

Sec. 3.1.2 pre-filters by depositing onto a grid of twice the target
resolution (TSC, 1024^3 for a 512^3 target), then applies the ideal discrete
low-pass filter and samples the filtered field at the target resolution.

Readings taken here (the paper does not spell these out):

* the ideal low-pass keeps the modes with |m_a| < N/2 on every axis (a cube in
  index space) and drops the target Nyquist planes m_a = -N/2;
* no assignment-window deconvolution is applied (none is mentioned);
* the result is normalised so that it sums to the deposited mass
  (numpy's unnormalised forward / 1/M inverse convention with M = N^3).
"""
from __future__ import annotations

import numpy as np

from .deposit import deposit, scheme_unit, galaxy_stencils


def crop_spectrum(gk, n):
    """Map a fine half spectrum (2n,2n,n+1) to the coarse half spectrum
    (n,n,n/2+1), keeping |m| < n/2 on every axis, zeros elsewhere."""
    nf = gk.shape[0]
    h = n // 2
    out = np.zeros((n, n, h + 1), dtype=np.complex128)
    keep_f = np.r_[0:h, nf - h + 1:nf]       # signed m in (-n/2, n/2)
    keep_c = np.r_[0:h, n - h + 1:n]
    out[np.ix_(keep_c, keep_c, np.arange(h))] = gk[np.ix_(keep_f, keep_f, np.arange(h))]
    return out


def lowpass_decimate(g_fine, n, workers=None):
    """Real fine field (2n)^3 -> band-limited real field n^3.  `workers`:
    scipy's FFT on that many threads (the same transform as numpy's)."""
    if workers:
        import scipy.fft as sf
        gk = sf.rfftn(g_fine, workers=workers)
        return sf.irfftn(crop_spectrum(gk, n), s=(n, n, n), axes=(0, 1, 2), workers=workers)
    gk = np.fft.rfftn(g_fine)
    return np.fft.irfftn(crop_spectrum(gk, n), s=(n, n, n), axes=(0, 1, 2))


def observed_counts(xyz, n, box, scheme, supersample, workers=None):
    """n^o on the n^3 target grid, plus the integer deposit it came from.

    supersample = 1: the deposit itself (times its unit).
    supersample = 2: deposit on (2n)^3, ideal low-pass, resample at n^3.
    """
    n_d = supersample * n
    grid = deposit(xyz, n_d, box, scheme)
    g = grid.astype(np.float64) * scheme_unit(scheme)
    if supersample == 1:
        return g, grid
    if supersample != 2:
        raise ValueError("supersample must be 1 or 2")
    return lowpass_decimate(g, n, workers), grid


def lowpass_kernel_1d(t, n):
    """D(t) = (1/n) sum_{|m| < n/2} exp(2 pi i m t / (2n)) for integer t: the
    1D impulse response of crop-then-resample from the 2n grid to the n grid."""
    t = np.asarray(t, dtype=np.float64)
    m = np.arange(1, n // 2, dtype=np.float64)
    return (1.0 + 2.0 * np.cos(np.pi * np.multiply.outer(t, m) / n).sum(axis=-1)) / n


def observed_counts_at(xyz, n, box, scheme, cells, chunk=1 << 16):
    """n^o at listed target cells by direct summation over every galaxy's
    stencil nodes f: n^o(j) = sum_f G(f) unit prod_a D(2 j_a - f_a).
    Independent of the FFT route; usable at any grid size."""
    cells = np.asarray(cells, dtype=np.int64).reshape(-1, 3)
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    n_d = 2 * n
    unit = scheme_unit(scheme)
    out = np.zeros(len(cells), dtype=np.float64)
    # D depends on (2 j - f) mod 2n only; tabulate once.
    dtab = lowpass_kernel_1d(np.arange(n_d), n)
    for lo in range(0, xyz.shape[0], chunk):
        idx, wt = galaxy_stencils(xyz[lo:lo + chunk], n_d, box, scheme)
        fz = idx % n_d
        fy = (idx // n_d) % n_d
        fx = idx // (n_d * n_d)
        wv = wt.astype(np.float64) * unit
        for c, (jx, jy, jz) in enumerate(cells):
            kx = dtab[(2 * jx - fx) % n_d]
            ky = dtab[(2 * jy - fy) % n_d]
            kz = dtab[(2 * jz - fz) % n_d]
            out[c] += np.dot(wv, kx * ky * kz)
    return out
