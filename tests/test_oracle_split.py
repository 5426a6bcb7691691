"""Pins of the oracle's prior-split system (C A C) y = C b, s = C y, with C the
square root of the prior covariance S (Sec. 3.3.1: S is diagonal in Fourier
space with eigenvalues P/dV)."""
import math

import numpy as np
import pytest

from oracle import wiener as ow
import synth


def _problem(n, box, seed, zero_frac=0.3, w_const=None):
    rng = np.random.Generator(np.random.PCG64(seed))
    ptab = synth.p_by_m2(lambda k: synth.bbks_power(k), n, box)
    if w_const is None:
        w = rng.uniform(0.1, 1.0, size=(n, n, n))
        w[rng.uniform(size=w.shape) < zero_frac] = 0.0
    else:
        w = np.full((n, n, n), float(w_const))
    nbar = 0.7
    b = np.where(w > 0, rng.standard_normal((n, n, n)), 0.0)
    return ptab, w, nbar, b


def _dft3(n):
    j = np.arange(n)
    f1 = np.exp(-2j * np.pi * np.outer(j, j) / n)
    return np.kron(np.kron(f1, f1), f1)


def _full_m2(n):
    j = np.arange(n)
    m = np.where(j < n // 2, j, j - n)
    return (m[:, None, None] ** 2 + m[None, :, None] ** 2 + m[None, None, :] ** 2).ravel()


def _dense(op, n):
    """Matrix of a linear map on n^3 fields, column by column."""
    M = n ** 3
    cols = []
    for i in range(M):
        e = np.zeros(M)
        e[i] = 1.0
        cols.append(op(e.reshape(n, n, n)).ravel())
    return np.array(cols).T


def test_split_operator_is_c_a_c_from_explicit_dft():
    """C A C from the oracle equals the product of dense matrices built from
    explicit DFT matrices and the prior's eigenvalues P/dV taken straight from
    the power table (no rfft, no Lambda table)."""
    n, box = 6, 40.0
    ptab, w, nbar, _ = _problem(n, box, seed=11)
    sysm = ow.System(n, box, w, ptab, nbar)
    sp = ow.SplitSystem(sysm)
    f3 = _dft3(n)
    M = n ** 3
    m2 = _full_m2(n)
    dv = (box / n) ** 3
    s_eig = np.where(m2 == 0, ptab[1] / dv, ptab[m2] / dv)  # monopole: value at |m|^2 = 1
    c_dense = ((f3.conj().T @ (np.sqrt(s_eig)[:, None] * f3)) / M).real
    a_dense = _dense(sysm.apply, n)
    want = c_dense @ a_dense @ c_dense
    got = _dense(sp.apply, n)
    assert np.abs(got - want).max() < 1e-10 * np.abs(want).max()
    # symmetric, and equal to I - P0 + C (nbar W) C
    assert np.abs(got - got.T).max() < 1e-10 * np.abs(got).max()
    p0 = np.full((M, M), 1.0 / M)
    alt = np.eye(M) - p0 + c_dense @ np.diag(nbar * w.ravel()) @ c_dense
    assert np.abs(got - alt).max() < 1e-10 * np.abs(alt).max()


def test_split_spectrum_bounds():
    """Eigenvalues of C A C lie in (0, 1 + nbar max(w) max(P/dV)], and all but
    the monopole direction are >= 1."""
    n, box = 6, 40.0
    ptab, w, nbar, _ = _problem(n, box, seed=12)
    sp = ow.SplitSystem(ow.System(n, box, w, ptab, nbar))
    ev = np.linalg.eigvalsh(_dense(sp.apply, n))
    pmax = (ptab[1:] / (box / n) ** 3).max()
    assert ev.min() > 0
    assert ev.max() <= 1 + nbar * w.max() * pmax * (1 + 1e-12)
    assert np.sort(ev)[1] >= 1 - 1e-10


def test_split_cg_solves_the_original_system():
    n, box = 16, 100.0
    ptab, w, nbar, b = _problem(n, box, seed=13)
    sysm = ow.System(n, box, w, ptab, nbar)
    ref = ow.reference_solution(sysm, b, 1e-13)["x"]
    res = ow.split_cg(sysm, b, 1e-12, 5000)
    assert res["status"] == "ok"
    assert ow.error_l2(res["x"], ref) < 1e-10
    assert res["rel_res_true"] < 1e-9


def test_split_cg_unmasked_closed_form():
    """w = const: A is diagonal in Fourier space, s_m = b_m / (Lambda_m + nbar w),
    and CG on C A C ends within the number of distinct eigenvalues."""
    n, box = 8, 60.0
    ptab, w, nbar, b = _problem(n, box, seed=14, w_const=0.8)
    sysm = ow.System(n, box, w, ptab, nbar)
    res = ow.split_cg(sysm, b, 1e-13, 500)
    want = np.fft.irfftn(np.fft.rfftn(b) / (sysm.lam + nbar * 0.8), s=b.shape, axes=(0, 1, 2))
    assert ow.error_l2(res["x"], want) < 1e-11
    n_distinct = len(np.unique(ow.m2_half_grid(n)))
    assert res["iterations"] <= n_distinct + 1


def test_split_cg_iterates_equal_prior_preconditioned_cg():
    """CG on C A C from y = 0 and preconditioned CG on A with M^-1 = S (the
    prior covariance, applied as one Fourier-diagonal product) produce the same
    iterates s_k = C y_k."""
    n, box = 16, 100.0
    ptab, w, nbar, b = _problem(n, box, seed=15)
    sysm = ow.System(n, box, w, ptab, nbar)
    c2 = ow.prior_split_factor(sysm) ** 2
    K = 12
    x = np.zeros_like(b)
    r = b.copy()
    z = np.fft.irfftn(c2 * np.fft.rfftn(r), s=b.shape, axes=(0, 1, 2))
    p = z.copy()
    rz = float(np.vdot(r, z))
    for _ in range(K):
        q = sysm.apply(p)
        a = rz / float(np.vdot(p, q))
        x += a * p
        r -= a * q
        z = np.fft.irfftn(c2 * np.fft.rfftn(r), s=b.shape, axes=(0, 1, 2))
        rz2 = float(np.vdot(r, z))
        p = z + (rz2 / rz) * p
        rz = rz2
    res = ow.split_cg(sysm, b, 0.0, K)
    assert res["iterations"] == K
    assert ow.error_l2(res["x"], x) < 1e-10


def test_split_cg_fewer_iterations_than_plain_on_a_masked_prior():
    """The point of the split: on a survey-like problem (cap mask, BBKS prior)
    it reaches the same residual in fewer iterations than plain CG."""
    wl = synth.workload("bbks512", n=24)
    ptab = wl.ptab()
    w = wl.mask()
    rng = np.random.Generator(np.random.PCG64(16))
    b = np.where(w > 0, rng.poisson(2.0, size=w.shape) - 2.0 * w, 0.0)
    sysm = ow.System(wl.n, wl.box, w, ptab, 2.0)
    plain = ow.cg(sysm, b, 1e-8, 20000)
    split = ow.split_cg(sysm, b, 1e-8, 20000)
    assert plain["status"] == split["status"] == "ok"
    assert split["iterations"] < plain["iterations"]
    assert ow.error_l2(split["x"], plain["x"]) < 1e-5
