"""The Wiener-filter system and its conjugate-gradient solve (oracle; test
infrastructure only).

The filter is the signal-space form of eq:WF (Sec. 3.3.1),

    <delta> = (S^-1 + W^T N^-1 W)^-1 W^T N^-1 delta^o,

with W = diag(w) the 3D completeness (Sec. 3.1.3, eq:RO with no bias or
redshift-space operator), the LSQ noise N = diag(w / nbar) (eq:noiseav), the
data delta^o = n^o/nbar - w (eq:datamodel) and nbar the fair-sample mean density
(eq:nmean).  S is diagonal in Fourier space with eigenvalues given by the prior
spectrum (Sec. 3.3.1, the Fourier representation of S_g,s).  Multiplying the
system by nbar gives the SPD problem solved here, in per-cell units:

    A s = b,   A = F^-1 diag(Lambda) F + diag(nbar w),
    b_i = n^o_i - nbar w_i  where w_i > 0,   0 where w_i = 0,
    Lambda_m = dV / P(k_m)  (m != 0),   Lambda_0 = 0.

Readings taken here: delta_D -> delta_ij / dV, so S has eigenvalues P/dV and
N_ii = w_i / nbar_cell; the k = 0 mode of S^-1 is 0 (a flat prior on the
monopole); nbar uses the integer input count; cells with w = 0 carry no data
and no noise term (Sec. 5.4: the noise term vanishes there and the filter
extrapolates into them).  The paper's Krylov method is not specified beyond
"iterative Krylov-space inversion" (Sec. 1); plain conjugate gradients from
x_0 = 0, stopped on the recursive relative residual ||r||/||b||, is the
reading used.
"""
from __future__ import annotations

import math

import numpy as np


def mean_density(n_gal, w):
    """eq:nmean in per-cell units: nbar = N_gal / sum_i w_i."""
    sw = float(np.sum(w, dtype=np.float64))
    if not sw > 0.0:
        raise ValueError("mask sums to zero")
    return float(n_gal) / sw


def data_vector(n_obs, w, nbar):
    """W^T N^-1 delta^o times nbar (eq:datamodel, eq:noiseav): n^o - nbar w on
    observed cells, 0 where w = 0."""
    return np.where(w > 0, n_obs - nbar * w, 0.0)


def lambda_table(p_by_m2, box, n):
    """Lambda_j = dV / P_j for j >= 1 (P tabulated at k = 2 pi sqrt(j) / L),
    Lambda_0 = 0 (Sec. 3.3.1, S diagonal in Fourier space)."""
    p = np.asarray(p_by_m2, dtype=np.float64)
    dv = (box / n) ** 3
    lam = np.zeros_like(p)
    lam[1:] = dv / p[1:]
    return lam


def m2_half_grid(n):
    """|m|^2 on numpy's rfftn layout (n, n, n/2+1), signed m in [-n/2, n/2)."""
    m = np.fft.fftfreq(n, 1.0 / n).astype(np.int64)
    mz = np.arange(n // 2 + 1, dtype=np.int64)
    return m[:, None, None] ** 2 + m[None, :, None] ** 2 + mz[None, None, :] ** 2


class System:
    """A s = b on an n^3 periodic grid (see the module docstring)."""

    def __init__(self, n, box, w, p_by_m2, nbar, workers=None):
        self.n = n
        self.box = box
        self.w = np.asarray(w, dtype=np.float64)
        self.nbar = float(nbar)
        self.nw = self.nbar * self.w
        self.lam = lambda_table(p_by_m2, box, n)[m2_half_grid(n)]
        self.workers = workers

    def _rfft(self, v):
        if self.workers:
            import scipy.fft as sf
            return sf.rfftn(v, workers=self.workers)
        return np.fft.rfftn(v)

    def _irfft(self, vk):
        s = (self.n,) * 3
        if self.workers:
            import scipy.fft as sf
            return sf.irfftn(vk, s=s, axes=(0, 1, 2), workers=self.workers)
        return np.fft.irfftn(vk, s=s, axes=(0, 1, 2))

    def apply(self, v):
        """A v = F^-1 Lambda F v + nbar w v (eq:WF, eq:noiseav)."""
        return self._irfft(self.lam * self._rfft(v)) + self.nw * v

    def precondition(self, r):
        """Fourier-diagonal approximate inverse (Lambda + nbar <w>)^-1, used only
        to reach reference solutions in fewer iterations."""
        d = self.lam + self.nbar * float(self.w.mean())
        return self._irfft(self._rfft(r) / d)


def cg(system, b, tol, max_iter, record=None, keep=()):
    """Plain conjugate gradients (Hestenes-Stiefel) from x_0 = 0.

    Stops after the first iteration whose recursive residual satisfies
    ||r|| / ||b|| <= tol, or after max_iter iterations.  Returns a dict with
    x, iterations, the recursive and true relative residuals, a status string
    and the CG coefficients (for Lanczos estimates); `kept` maps every
    iteration count listed in `keep` that was reached to a copy of that
    iterate (an observation only: the arithmetic is the same with or without).
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    bnorm = math.sqrt(float(np.vdot(b, b)))
    kept = {}
    if bnorm == 0.0:
        return dict(x=x, iterations=0, rel_res=0.0, rel_res_true=0.0,
                    status="ok", alphas=[], betas=[], kept=kept)
    r = b.copy()
    p = r.copy()
    rho = float(np.vdot(r, r))
    alphas, betas = [], []
    status = "maxiter"
    it = 0
    rel = 1.0
    while it < max_iter:
        q = system.apply(p)
        pq = float(np.vdot(p, q))
        if not (pq > 0.0) or not math.isfinite(pq):
            status = "breakdown"
            break
        alpha = rho / pq
        x += alpha * p
        r -= alpha * q
        rho_new = float(np.vdot(r, r))
        it += 1
        alphas.append(alpha)
        rel = math.sqrt(rho_new) / bnorm
        if record is not None:
            record.append(rel)
        if it in keep:
            kept[it] = x.copy()
        if rel <= tol:
            status = "ok"
            break
        beta = rho_new / rho
        betas.append(beta)
        rho = rho_new
        p = r + beta * p
    rt = b - system.apply(x)
    return dict(x=x, iterations=it, rel_res=rel,
                rel_res_true=math.sqrt(float(np.vdot(rt, rt))) / bnorm,
                status=status, alphas=alphas, betas=betas, kept=kept)


def pcg(system, b, tol, max_iter):
    """Preconditioned CG with system.precondition; same solution A^-1 b as cg,
    used to produce reference solutions.  Stops on the true-ish recursive
    residual ||r|| / ||b||."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    bnorm = math.sqrt(float(np.vdot(b, b)))
    if bnorm == 0.0:
        return dict(x=x, iterations=0, rel_res=0.0)
    r = b.copy()
    z = system.precondition(r)
    p = z.copy()
    rz = float(np.vdot(r, z))
    it = 0
    rel = 1.0
    while it < max_iter:
        q = system.apply(p)
        alpha = rz / float(np.vdot(p, q))
        x += alpha * p
        r -= alpha * q
        it += 1
        rel = math.sqrt(float(np.vdot(r, r))) / bnorm
        if rel <= tol:
            break
        z = system.precondition(r)
        rz_new = float(np.vdot(r, z))
        p = z + (rz_new / rz) * p
        rz = rz_new
    return dict(x=x, iterations=it, rel_res=rel)


def prior_split_factor(system):
    """c_m of the prior split C = F^-1 diag(c) F on the half-spectrum grid:
    c_m = Lambda_m^(-1/2) = (P(k_m)/dV)^(1/2), the square root of the prior's
    Fourier eigenvalues (Sec. 3.3.1).  Lambda_0 = 0 (flat monopole prior) has
    no root; c_0 takes the value of the |m|^2 = 1 modes, which keeps the
    monopole's eigenvalue of C A C inside the range of the others."""
    lam = system.lam
    c = np.zeros_like(lam)
    pos = lam > 0
    c[pos] = 1.0 / np.sqrt(lam[pos])
    m2 = m2_half_grid(system.n)
    c[~pos] = 1.0 / math.sqrt(float(lam[m2 == 1][0]))
    return c


class SplitSystem:
    """The Wiener system preconditioned by its prior on both sides:
    (C A C) y = C b with s = C y.  C is symmetric positive definite, so the
    solution s = A^-1 b is the one of the plain system; C A C equals
    I - P_0 + C diag(nbar w) C (P_0 the projection on the constant field)
    and has its spectrum in [min(1, .), 1 + nbar max(w) max(P/dV)], whereas
    the spectrum of A spans the whole range of Lambda.  Written here as the
    literal product of the three operators."""

    def __init__(self, system):
        self.base = system
        self.c = prior_split_factor(system)

    def split(self, v):
        """C v."""
        return self.base._irfft(self.c * self.base._rfft(v))

    def apply(self, y):
        """(C A C) y."""
        return self.split(self.base.apply(self.split(y)))


def split_cg(system, b, tol, max_iter, record=None):
    """Plain CG (the cg above) on the prior-split system from y_0 = 0,
    stopped on its own recursive residual ||r_y|| / ||C b|| <= tol; returns
    the solution s = C y together with the split run's numbers and the true
    residual of the original system ||b - A s|| / ||b||."""
    sp = SplitSystem(system)
    b = np.asarray(b, dtype=np.float64)
    res = cg(sp, sp.split(b), tol, max_iter, record=record)
    s = sp.split(res["x"])
    bnorm = math.sqrt(float(np.vdot(b, b)))
    rt = b - system.apply(s)
    out = dict(res)
    out.update(y=res["x"], x=s, rel_res_split=res["rel_res"],
               rel_res_true=(math.sqrt(float(np.vdot(rt, rt))) / bnorm) if bnorm > 0 else 0.0)
    return out


def reference_solution(system, b, tol=1e-13, max_iter=20000):
    """A^-1 b to a tight tolerance (PCG), for error measurements."""
    return pcg(system, b, tol, max_iter)


def lanczos_extremes(alphas, betas):
    """Ritz values of A from CG coefficients (tridiagonal Lanczos matrix):
    T_jj = 1/a_j + b_{j-1}/a_{j-1}, T_j,j+1 = sqrt(b_j)/a_j."""
    k = len(alphas)
    if k == 0:
        return float("nan"), float("nan")
    a = np.asarray(alphas)
    bb = np.asarray(betas[:k - 1]) if k > 1 else np.zeros(0)
    diag = 1.0 / a
    diag[1:] += bb / a[:-1]
    off = np.sqrt(bb) / a[:-1]
    t = np.diag(diag) + np.diag(off, 1) + np.diag(off, -1)
    ev = np.linalg.eigvalsh(t)
    return float(ev[0]), float(ev[-1])


def error_l2(x, x_ref):
    """||x - x_ref||_2 / ||x_ref||_2 over all cells."""
    x = np.asarray(x, dtype=np.float64)
    d = x - x_ref
    return math.sqrt(float(np.vdot(d, d)) / float(np.vdot(x_ref, x_ref)))


def reconstruct(xyz, n, box, w, p_by_m2, scheme, supersample, tol, max_iter,
                workers=None):
    """The whole path: deposit -> n^o -> nbar, b -> CG solve."""
    from .supersample import observed_counts
    n_obs, grid = observed_counts(xyz, n, box, scheme, supersample)
    nbar = mean_density(len(xyz), w)
    b = data_vector(n_obs, w, nbar)
    system = System(n, box, w, p_by_m2, nbar, workers=workers)
    res = cg(system, b, tol, max_iter)
    res.update(n_obs=n_obs, grid=grid, nbar=nbar, b=b, system=system)
    return res
