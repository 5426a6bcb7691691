"""Seeded synthetic inputs for the Wiener reconstruction (shared by the oracle
side and the HIP side as *data*; this module holds none of the filter's own
arithmetic: no Fourier diagonal, no data vector, no operator, no solve).

The paper reconstructs SDSS DR6 galaxies (Sec. 2) and validates on a
Millennium-based mock (Sec. 4); neither catalogue is available, so these
generators stand in for them with catalogues of the same structure:

* a prior power spectrum P(k) -- a power law with a Gaussian cut-off, or a
  CDM-like BBKS transfer function normalised to sigma_8 -- tabulated on the
  integer |m|^2 lattice that a periodic N^3 grid of side L samples
  (k = 2 pi sqrt(j) / L);
* a 3D completeness w(s) <= 1: a spherical sky cap seen from an observer times
  a radial selection exp(-r/r0) (Sec. 3.1.3 builds w as sky completeness times
  radial selection);
* a lognormal density field (Sec. 5.5 finds the reconstructed density close
  to lognormal) Poisson-sampled with mean w * lambda, which is the
  Poisson-binomial observation law of Sec. 3.2.2 (eq:poisbin, eq:poisbinmean);
* galaxy positions uniform inside their node-centred cell, wrapped into the
  periodic box [0, L).

Everything is drawn from numpy's PCG64 with explicit seeds.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# Cosmology of Sec. 3.1.1: Omega_m = 0.24, Omega_Lambda = 0.76, Omega_K = 0,
# H0 = 100 h km/s/Mpc with h = 0.73 (the text prints "h=73").
OMEGA_M = 0.24
HUBBLE_H = 0.73


# ---------------------------------------------------------------------------
# P(k) models.  k is in 1/Mpc, P in Mpc^3.
# ---------------------------------------------------------------------------

def power_law_shape(k):
    """Unnormalised power law P = k_h^-1.5 exp(-(k_h/0.5)^2), k_h = k/h in h/Mpc,
    returned in Mpc^3 (a (Mpc/h)^3 spectrum divided by h^3)."""
    k = np.asarray(k, dtype=np.float64)
    kh = k / HUBBLE_H
    with np.errstate(divide="ignore"):
        p = np.where(kh > 0, kh ** -1.5 * np.exp(-(kh / 0.5) ** 2), 0.0)
    return p / HUBBLE_H ** 3


def bbks_transfer(q):
    """BBKS (Bardeen, Bond, Kaiser & Szalay 1986) CDM transfer function of
    q = k_h / Gamma."""
    q = np.asarray(q, dtype=np.float64)
    out = np.ones_like(q)
    nz = q > 0
    x = q[nz]
    out[nz] = (np.log1p(2.34 * x) / (2.34 * x)
               * (1.0 + 3.89 * x + (16.1 * x) ** 2 + (5.46 * x) ** 3
                  + (6.71 * x) ** 4) ** -0.25)
    return out


def _tophat(x):
    x = np.asarray(x, dtype=np.float64)
    small = x < 1e-4
    xs = np.where(small, 1.0, x)
    w = 3.0 * (np.sin(xs) - xs * np.cos(xs)) / xs ** 3
    return np.where(small, 1.0 - x * x / 10.0, w)


def bbks_power(k, n_s=0.96, sigma8=0.8, omega_m=OMEGA_M, h=HUBBLE_H, amp=1.0):
    """CDM-like linear spectrum P = A k_h^n_s T^2(k_h/Gamma), Gamma = Omega_m h,
    normalised so that sigma_8 (top hat of 8 Mpc/h) equals `sigma8`; times
    `amp` (the serving workload varies it by +-20%).  Mpc^3."""
    gamma = omega_m * h
    kk = np.logspace(-5, 3, 40001)  # h/Mpc
    pk = kk ** n_s * bbks_transfer(kk / gamma) ** 2
    integrand = kk ** 3 * pk * _tophat(kk * 8.0) ** 2 / (2 * math.pi ** 2)
    s2 = np.trapezoid(integrand, np.log(kk))
    norm = sigma8 ** 2 / s2
    k = np.asarray(k, dtype=np.float64)
    kh = k / h
    p = norm * kh ** n_s * bbks_transfer(kh / gamma) ** 2  # (Mpc/h)^3
    return amp * p / h ** 3


def m2_table_len(n):
    """Number of distinct integer |m|^2 values on an n^3 periodic grid: 3(n/2)^2+1."""
    return 3 * (n // 2) ** 2 + 1


def p_by_m2(pfun, n, box):
    """Tabulate P at k = 2 pi sqrt(j)/L for j = 0 .. 3(n/2)^2.  Entry 0 is set
    to 0 (the k = 0 entry is not used by the filter)."""
    j = np.arange(m2_table_len(n), dtype=np.float64)
    k = 2.0 * math.pi * np.sqrt(j) / box
    p = np.asarray(pfun(k), dtype=np.float64)
    p[0] = 0.0
    return p


def _m2_grid(n):
    m = np.fft.fftfreq(n, 1.0 / n).astype(np.int64)
    mz = np.arange(n // 2 + 1, dtype=np.int64)
    return m[:, None, None] ** 2 + m[None, :, None] ** 2 + mz[None, None, :] ** 2


def cell_variance(ptab, n, box):
    """Per-cell Gaussian variance (1/M) sum_{m != 0} P(k_m)/dV of a field with
    spectrum `ptab` (indexed by |m|^2) on an n^3 grid (full-spectrum count)."""
    dv = (box / n) ** 3
    m2 = _m2_grid(n)
    pc = ptab[m2] / dv
    pc[0, 0, 0] = 0.0
    wgt = np.full(pc.shape, 2.0)
    wgt[..., 0] = 1.0
    if n % 2 == 0:
        wgt[..., n // 2] = 1.0
    return float((wgt * pc).sum() / n ** 3)


def power_law_normalised(n=32, box=256.0, sigma_g2=0.5):
    """Power law scaled so that its per-cell Gaussian variance on the n^3 grid
    of side `box` is `sigma_g2` (0.5 for the 32^3 / 256 Mpc workload)."""
    base = p_by_m2(power_law_shape, n, box)
    amp = sigma_g2 / cell_variance(base, n, box)
    return lambda k: amp * power_law_shape(k)


# ---------------------------------------------------------------------------
# Masks: spherical cap times radial selection.
# ---------------------------------------------------------------------------

def cap_mask(n, box, theta_deg=60.0, r0=150.0, axis=(0.0, 0.0, 1.0),
             observer=None):
    """w at nodes x_n = n H: inside the cap (angle to `axis` <= theta, inclusive,
    and r <= L/2) w = exp(-r/r0), else 0; w = 1 at the observer.  The observer
    defaults to node (n/2)(1,1,1)."""
    h = box / n
    if observer is None:
        observer = np.full(3, (n // 2) * h)
    ax = np.asarray(axis, dtype=np.float64)
    ax = ax / np.linalg.norm(ax)
    c = np.arange(n, dtype=np.float64) * h
    dx = c[:, None, None] - observer[0]
    dy = c[None, :, None] - observer[1]
    dz = c[None, None, :] - observer[2]
    r = np.sqrt(dx * dx + dy * dy + dz * dz)
    dot = dx * ax[0] + dy * ax[1] + dz * ax[2]
    cos_t = math.cos(math.radians(theta_deg))
    with np.errstate(invalid="ignore", divide="ignore"):
        inside = (dot >= cos_t * r) & (r <= box / 2)
    w = np.where(inside, np.exp(-r / r0), 0.0)
    w[r == 0] = 1.0
    return np.ascontiguousarray(w)


def random_axis(rng):
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


# ---------------------------------------------------------------------------
# Lognormal-Poisson catalogues.
# ---------------------------------------------------------------------------

def gaussian_field(ptab, n, box, seed):
    """Gaussian random field with spectrum P (per-cell units P/dV), zero mean
    mode, built by colouring white noise in Fourier space.  Uses scipy's FFT on
    all host cores (its result does not depend on the thread count)."""
    import scipy.fft as sf
    rng = np.random.Generator(np.random.PCG64(seed))
    eps = rng.standard_normal((n, n, n))
    dv = (box / n) ** 3
    amp = np.sqrt(ptab[_m2_grid(n)] / dv)
    amp[0, 0, 0] = 0.0
    ek = sf.rfftn(eps, workers=-1)
    del eps
    ek *= amp
    return sf.irfftn(ek, s=(n, n, n), axes=(0, 1, 2), workers=-1)


def lognormal_density(ptab, n, box, seed):
    """1 + delta = exp(g - sigma_G^2/2), sigma_G^2 = the per-cell variance."""
    g = gaussian_field(ptab, n, box, seed)
    s2 = cell_variance(ptab, n, box)
    return np.exp(g - 0.5 * s2), s2


def poisson_binomial_two_stage(lam, w, rng):
    """Eq:pois then eq:bin: N ~ Poisson(lambda), N_o ~ Binomial(N, w)."""
    full = rng.poisson(lam)
    return rng.binomial(full, w)


def poisson_direct(lam, w, rng):
    """Eq:poisbin: N_o ~ Poisson(w lambda)."""
    return rng.poisson(w * lam)


@dataclass
class Catalogue:
    xyz: np.ndarray          # (n_gal, 3) float64, Mpc, in [0, L)
    counts: np.ndarray       # (n, n, n) int64 galaxies per generator cell
    one_plus_delta: np.ndarray
    sigma_g2: float


def lognormal_catalogue(ptab, w, box, n_target, seed, rate_scale=None):
    """Counts N_i ~ Poisson(n_in (1+delta_i) w_i) with n_in chosen so that
    sum lambda = n_target; positions uniform in the node-centred cell
    [(n-1/2)H, (n+1/2)H), wrapped into [0, L).  Seeds: field `seed`,
    counts `seed+1`, positions `seed+2`."""
    n = w.shape[0]
    opd, s2 = lognormal_density(ptab, n, box, seed)
    lam = opd * w
    tot = lam.sum()
    if tot <= 0:
        raise ValueError("mask selects nothing")
    lam *= n_target / tot
    counts = np.random.Generator(np.random.PCG64(seed + 1)).poisson(lam)
    xyz = place_in_cells(counts, box, seed + 2)
    return Catalogue(xyz=xyz, counts=counts, one_plus_delta=opd, sigma_g2=s2)


def place_in_cells(counts, box, seed):
    n = counts.shape[0]
    h = box / n
    rng = np.random.Generator(np.random.PCG64(seed))
    flat = counts.ravel()
    idx = np.repeat(np.arange(flat.size, dtype=np.int64), flat)
    ix, iy, iz = np.unravel_index(idx, counts.shape)
    base = np.stack([ix, iy, iz], axis=1).astype(np.float64)
    off = rng.uniform(-0.5, 0.5, size=base.shape)
    xyz = (base + off) * h
    xyz = np.mod(xyz, box)
    xyz[xyz >= box] = 0.0  # mod can round up to exactly box
    return np.ascontiguousarray(xyz)


def uniform_catalogue(n_gal, box, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    xyz = rng.uniform(0.0, box, size=(n_gal, 3))
    xyz[xyz >= box] = 0.0
    return np.ascontiguousarray(xyz)


# ---------------------------------------------------------------------------
# The workloads (grid, box, spectrum, mask, catalogue size, deposit scheme).
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    n: int
    box: float
    scheme: str           # "ngp" | "cic" | "tsc"
    supersample: int
    n_target: int
    seed: int
    spectrum: str         # "powerlaw" | "bbks"
    theta_deg: float = 60.0
    r0: float = 150.0
    amp: float = 1.0
    axis: tuple = (0.0, 0.0, 1.0)

    def ptab(self):
        if self.spectrum == "powerlaw":
            f = power_law_normalised(32, 256.0, 0.5)
        else:
            amp = self.amp
            f = lambda k: bbks_power(k, amp=amp)  # noqa: E731
        return p_by_m2(f, self.n, self.box)

    def mask(self):
        return cap_mask(self.n, self.box, self.theta_deg, self.r0, self.axis)

    def catalogue(self, ptab=None, w=None):
        ptab = self.ptab() if ptab is None else ptab
        w = self.mask() if w is None else w
        return lognormal_catalogue(ptab, w, self.box, self.n_target, self.seed)


def workload(name, seed=None, n=None):
    """Named workloads.  `n` rescales the grid (same box and recipe)."""
    table = {
        # 32^3 / 256 Mpc, power law, NGP, FP64, residual 1e-10
        "pl32": Workload("pl32", 32, 256.0, "ngp", 1, 20000, 101, "powerlaw"),
        # 256^3 / 500 Mpc, BBKS, 2x supersampled CIC, FP64, residual 1e-6
        "bbks256": Workload("bbks256", 256, 500.0, "cic", 2, 1_000_000, 201, "bbks"),
        # 512^3 / 500 Mpc, BBKS, 2x supersampled TSC, mixed, error <= 1e-6
        "bbks512": Workload("bbks512", 512, 500.0, "tsc", 2, 500_000, 301, "bbks"),
    }
    wl = table[name]
    if seed is not None:
        wl.seed = seed
    if n is not None:
        wl.n = n
    return wl


def serving_request(i, base_seed=5001, box=500.0, grids=(64, 128, 256, 384)):
    """Request i of the serving stream: grid uniform over `grids`, cap half
    angle U[30, 90] deg with an isotropic axis, r0 U[100, 250] Mpc, BBKS
    amplitude x U[0.8, 1.2], n_gal log-uniform in [1e4, 2e6], CIC with 2x
    supersampling."""
    seed = base_seed + 3 * i
    rng = np.random.Generator(np.random.PCG64(seed + 7))
    n = int(rng.choice(np.asarray(grids)))
    theta = float(rng.uniform(30.0, 90.0))
    r0 = float(rng.uniform(100.0, 250.0))
    amp = float(rng.uniform(0.8, 1.2))
    ngal = int(round(10 ** rng.uniform(4.0, math.log10(2e6))))
    axis = tuple(random_axis(rng))
    return Workload(f"req{i}", n, box, "cic", 2, ngal, seed, "bbks",
                    theta_deg=theta, r0=r0, amp=amp, axis=axis)
