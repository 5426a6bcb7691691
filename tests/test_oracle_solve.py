"""Pins of the oracle's Wiener system and CG solve (eq:WF with the LSQ noise of
eq:noiseav, Sec. 3.3.1)."""
import math

import numpy as np
import pytest

from oracle import wiener as ow
import synth


def _problem(n, box, seed, mask="random", zero_frac=0.3):
    rng = np.random.Generator(np.random.PCG64(seed))
    ptab = synth.p_by_m2(lambda k: synth.bbks_power(k), n, box)
    if mask == "random":
        w = rng.uniform(0.1, 1.0, size=(n, n, n))
        w[rng.uniform(size=w.shape) < zero_frac] = 0.0
    else:
        w = np.full((n, n, n), float(mask))
    nbar = 0.7
    b = np.where(w > 0, rng.standard_normal((n, n, n)), 0.0)
    return ptab, w, nbar, b


def _dense_operator(n, box, w, ptab, nbar):
    """A built from explicit DFT matrices (Kronecker product of 1D DFTs) and the
    full (not half) spectrum of S^-1; independent of the oracle's rfft route."""
    j = np.arange(n)
    f1 = np.exp(-2j * np.pi * np.outer(j, j) / n)
    f3 = np.kron(np.kron(f1, f1), f1)
    m = np.where(j < n // 2, j, j - n)  # signed
    m2 = (m[:, None, None] ** 2 + m[None, :, None] ** 2 + m[None, None, :] ** 2).ravel()
    dv = (box / n) ** 3
    lam = np.where(m2 == 0, 0.0, dv / np.where(m2 == 0, 1.0, ptab[m2]))
    M = n ** 3
    a = (f3.conj().T @ (lam[:, None] * f3)) / M
    assert np.abs(a.imag).max() < 1e-9 * np.abs(a.real).max()
    return a.real + np.diag(nbar * w.ravel())


@pytest.mark.parametrize("n", [8, 6])
def test_cg_matches_dense_cholesky(n):
    box = 40.0
    ptab, w, nbar, b = _problem(n, box, seed=n)
    A = _dense_operator(n, box, w, ptab, nbar)
    L = np.linalg.cholesky(A)
    y = np.linalg.solve(L, b.ravel())
    x_ref = np.linalg.solve(L.T, y)
    sysm = ow.System(n, box, w, ptab, nbar)
    res = ow.cg(sysm, b, 1e-14, 5000)
    assert res["status"] == "ok"
    assert ow.error_l2(res["x"].ravel(), x_ref) < 1e-12
    # the operator itself against the dense matrix
    v = np.random.Generator(np.random.PCG64(1)).standard_normal((n, n, n))
    assert np.allclose(sysm.apply(v).ravel(), A @ v.ravel(), rtol=0, atol=1e-12 * np.abs(A).max())


def test_lanczos_extremes_approach_dense_spectrum():
    n, box = 8, 40.0
    ptab, w, nbar, b = _problem(n, box, seed=3)
    A = _dense_operator(n, box, w, ptab, nbar)
    ev = np.linalg.eigvalsh(A)
    res = ow.cg(ow.System(n, box, w, ptab, nbar), b, 1e-14, 5000)
    lo, hi = ow.lanczos_extremes(res["alphas"], res["betas"])
    assert ev[0] * (1 - 1e-6) <= lo <= ev[0] * 1.01
    assert ev[-1] * 0.99 <= hi <= ev[-1] * (1 + 1e-6)


@pytest.mark.parametrize("c", [1.0, 0.37])
def test_closed_form_uniform_mask(c):
    """With w = c everywhere, A is diagonal in Fourier space:
    s_k = b_k / (Lambda_k + nbar c); for c = 1 this is the textbook Wiener
    filter s_k = P_k / (P_k + 1/nbar) d_k with d = b / nbar (per-cell P)."""
    n, box = 16, 300.0
    ptab, w, nbar, b = _problem(n, box, seed=5, mask=c)
    res = ow.cg(ow.System(n, box, w, ptab, nbar), b, 1e-14, 5000)
    # independent route: full complex FFT with Lambda on the full index grid
    m = np.fft.fftfreq(n, 1.0 / n)
    kk = 2 * np.pi / box * np.sqrt(m[:, None, None] ** 2 + m[None, :, None] ** 2
                                   + m[None, None, :] ** 2)
    dv = (box / n) ** 3
    pk = np.where(kk > 0, synth.bbks_power(np.where(kk > 0, kk, 1.0)), np.inf)
    pcell = pk / dv
    if c == 1.0:
        d = b / nbar
        noise = 1.0 / nbar
        with np.errstate(invalid="ignore"):
            filt = np.where(np.isinf(pcell), 1.0, pcell / (pcell + noise))
        s = np.fft.ifftn(filt * np.fft.fftn(d)).real
    else:
        lam = np.where(np.isinf(pcell), 0.0, 1.0 / pcell)
        s = np.fft.ifftn(np.fft.fftn(b) / (lam + nbar * c)).real
    assert ow.error_l2(res["x"], s) < 1e-12


def test_operator_symmetric_positive_and_solve_linear():
    n, box = 12, 100.0
    ptab, w, nbar, b = _problem(n, box, seed=7)
    sysm = ow.System(n, box, w, ptab, nbar)
    rng = np.random.Generator(np.random.PCG64(2))
    u = rng.standard_normal((n, n, n))
    v = rng.standard_normal((n, n, n))
    lhs = np.vdot(u, sysm.apply(v))
    rhs = np.vdot(sysm.apply(u), v)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs) * 10 + 1e-12
    assert np.vdot(u, sysm.apply(u)) > 0
    b2 = np.where(w > 0, rng.standard_normal((n, n, n)), 0.0)
    x1 = ow.cg(sysm, b, 1e-13, 4000)["x"]
    x2 = ow.cg(sysm, b2, 1e-13, 4000)["x"]
    x3 = ow.cg(sysm, 2.0 * b - 3.0 * b2, 1e-13, 4000)["x"]
    assert ow.error_l2(x3, 2.0 * x1 - 3.0 * x2) < 1e-10


def test_periodic_translation_covariance():
    n, box = 12, 100.0
    ptab, w, nbar, b = _problem(n, box, seed=8)
    sh = (3, -5, 7)
    x = ow.cg(ow.System(n, box, w, ptab, nbar), b, 1e-13, 4000)["x"]
    xs = ow.cg(ow.System(n, box, np.roll(w, sh, (0, 1, 2)), ptab, nbar),
               np.roll(b, sh, (0, 1, 2)), 1e-13, 4000)["x"]
    assert ow.error_l2(xs, np.roll(x, sh, (0, 1, 2))) < 1e-10


def test_unobserved_cells_carry_no_data():
    w = np.array([[[0.0, 0.5], [1.0, 0.0]]])
    n_obs = np.array([[[3.0, 2.0], [1.0, 4.0]]])
    b = ow.data_vector(n_obs, w, 2.0)
    assert b.tolist() == [[[0.0, 1.0], [-1.0, 0.0]]]


def test_mean_density_fair_sample():
    w = np.array([0.5, 0.25, 0.25, 0.0])
    assert ow.mean_density(10, w) == 10.0
    with pytest.raises(ValueError):
        ow.mean_density(3, np.zeros(4))


def test_lambda_table_zero_mode_and_units():
    p = np.array([0.0, 2.0, 4.0, 8.0])
    lam = ow.lambda_table(p, 10.0, 5)
    assert lam[0] == 0.0
    assert np.allclose(lam[1:], 8.0 / p[1:])


def test_cg_zero_rhs_and_maxiter_and_breakdown():
    n, box = 8, 40.0
    ptab, w, nbar, b = _problem(n, box, seed=9)
    sysm = ow.System(n, box, w, ptab, nbar)
    r0 = ow.cg(sysm, np.zeros_like(b), 1e-10, 10)
    assert r0["iterations"] == 0 and np.all(r0["x"] == 0)
    r1 = ow.cg(sysm, b, 0.0, 7)
    assert r1["iterations"] == 7 and r1["status"] == "maxiter"
    bad = ow.System(n, box, w, -ptab, nbar)  # negative prior -> indefinite
    bad.nw[:] = 0.0
    r2 = ow.cg(bad, b, 1e-10, 50)
    assert r2["status"] == "breakdown"


def test_pcg_reaches_same_solution():
    n, box = 16, 200.0
    ptab, w, nbar, b = _problem(n, box, seed=10)
    sysm = ow.System(n, box, w, ptab, nbar)
    x1 = ow.cg(sysm, b, 1e-13, 5000)["x"]
    x2 = ow.pcg(sysm, b, 1e-13, 5000)["x"]
    assert ow.error_l2(x2, x1) < 1e-11


def test_error_tracks_residual_on_workload_recipe():
    # 32^3 power-law workload: reaching residual 1e-10 gives an error
    # against the tight reference far below 1e-6.
    wl = synth.workload("pl32")
    ptab = wl.ptab()
    w = wl.mask()
    cat = wl.catalogue(ptab, w)
    res = ow.reconstruct(cat.xyz, wl.n, wl.box, w, ptab, "ngp", 1, 1e-10, 5000)
    assert res["status"] == "ok"
    assert res["rel_res_true"] < 1e-9
    ref = ow.reference_solution(res["system"], res["b"])
    assert ow.error_l2(res["x"], ref["x"]) < 1e-7
    assert math.isfinite(res["nbar"]) and res["nbar"] > 0
