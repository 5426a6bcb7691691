"""The algebra of the folded FP32 prior-split iteration, checked in FP64 on the
host against the oracle's textbook CG (the oracle itself stays textbook).

The folded iteration applies r -= alpha q at the start of the next iteration
(in the pass that forms the direction), so beta must come before the new
residual exists: with r.q = p.q (r and p differ by a multiple of the previous
direction, A-conjugate to p), |r - alpha q|^2 = alpha^2 q.q - r.r.  alpha and
the stopping tests use the exact r.r of the vector written.  A reliable update
continues the direction already formed with the refreshed residual,
p += r_new - r_old.  These tests restate that arithmetic and compare it with
cg() of oracle/wiener.py on the prior-split system (Sec. 3.3.1, eq:WF)."""
import math

import numpy as np
import pytest

import synth
from oracle import wiener as ow


def _split_problem(n=12, box=300.0, seed=11, nbar=200.0):
    """A 12^3 prior-split system whose CG needs ~60 iterations to 1e-12."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ptab = synth.p_by_m2(lambda k: synth.bbks_power(k), n, box)
    w = rng.uniform(0.2, 1.0, size=(n, n, n))
    w[rng.uniform(size=w.shape) < 0.4] = 0.0
    b = np.where(w > 0, rng.standard_normal((n, n, n)), 0.0)
    system = ow.System(n, box, w, ptab, nbar)
    sp = ow.SplitSystem(system)
    return sp, sp.split(b)


def folded_cg(op, b, iters, update_at=()):
    """The folded recurrence: each call of the loop body is one iteration of
    the GPU path (first pass: pending x and r updates, exact r.r, direction;
    then q = op(p), p.q and q.q; alpha and the recurrence beta).  With
    `update_at`, a reliable update (true residual b - op(x), direction
    continued) happens right after the first pass of those iteration counts.
    Returns x with the last step applied, the iteration count, the betas used
    and, per applied step, the recurrence's r.r beside the exact r.r of the
    residual written."""
    x = np.zeros_like(b)
    r = b.copy()
    p = np.zeros_like(b)
    q = np.zeros_like(b)
    rho = float(np.vdot(r, r))
    alpha = beta = 0.0
    pending, first = False, True
    done = 0
    betas, pairs = [], []
    rho_next = 0.0
    while True:
        # first pass
        if pending:
            x += alpha * p
            r -= alpha * q
            p = r + beta * p
            done += 1
        elif first:
            p = r.copy()
        rho = float(np.vdot(r, r))  # the exact r.r of what was written
        if pending:
            pairs.append((rho_next, rho))
        first, pending = False, False
        if done in update_at and done > 0:
            r_new = b - op(x)
            p += r_new - r
            r = r_new
            rho = float(np.vdot(r, r))
        if done >= iters:
            return x, done, betas, pairs
        # operator and the two dot products
        q = op(p)
        pq = float(np.vdot(p, q))
        qq = float(np.vdot(q, q))
        alpha = rho / pq
        rho_next = alpha * alpha * qq - rho
        beta = rho_next / rho if rho_next > 0.0 else 0.0
        betas.append(beta)
        pending = True


@pytest.mark.parametrize("k", [1, 5, 30, 50])
def test_folded_iterates_equal_textbook_cg(k):
    sp, b = _split_problem()
    ref = ow.cg(sp, b, 0.0, k, keep=(k,))
    x, done, _, _ = folded_cg(sp.apply, b, k)
    assert done == k
    err = np.linalg.norm(x - ref["kept"][k]) / np.linalg.norm(ref["kept"][k])
    assert err < 1e-10, err


def test_recurrence_rr_matches_the_exact_rr():
    """Within one folded run, alpha^2 q.q - r.r against the exact r.r of the
    residual the next pass writes, at every step down to a residual of
    1e-11; and the folded betas against the textbook run's over the first 30
    steps (later the two runs' coefficients part at rounding level, as any
    two CG runs that differ by rounding do once orthogonality is lost, while
    the iterates still agree: test_folded_iterates_equal_textbook_cg)."""
    sp, b = _split_problem()
    ref = ow.cg(sp, b, 1e-11, 500)
    _, _, betas, pairs = folded_cg(sp.apply, b, ref["iterations"])
    est, exact = np.asarray(pairs).T
    assert len(est) > 40
    assert np.max(np.abs(est / exact - 1.0)) < 1e-11
    tb = np.asarray(ref["betas"][:30])
    assert np.max(np.abs(np.asarray(betas[:30]) / tb - 1.0)) < 1e-12


def test_recurrence_beta_is_wrong_without_conjugacy():
    """A plausible slip (using r.q = 0 instead of p.q, i.e. rho_next =
    rho + alpha^2 q.q) is far off: the identity matters."""
    sp, b = _split_problem()
    r = b.copy()
    p = r.copy()
    q = sp.apply(p)
    rho = float(np.vdot(r, r))
    alpha = rho / float(np.vdot(p, q))
    exact = float(np.vdot(r - alpha * q, r - alpha * q))
    wrong = rho + alpha * alpha * float(np.vdot(q, q))
    right = alpha * alpha * float(np.vdot(q, q)) - rho
    assert abs(right / exact - 1.0) < 1e-10
    assert abs(wrong / exact - 1.0) > 0.5


def test_continued_direction_after_a_residual_replacement():
    """p += r_new - r_old after the direction was formed equals forming it
    from the replaced residual with the same beta; in exact arithmetic the
    true and recursive residuals agree, so the run equals textbook CG."""
    sp, b = _split_problem()
    ref = ow.cg(sp, b, 0.0, 45, keep=(45,))
    x, done, _, _ = folded_cg(sp.apply, b, 45, update_at=(10, 25, 40))
    err = np.linalg.norm(x - ref["kept"][45]) / np.linalg.norm(ref["kept"][45])
    assert done == 45 and err < 1e-9, err
    rng = np.random.Generator(np.random.PCG64(3))
    r_old, r_new, p_old = (rng.standard_normal(50) for _ in range(3))
    beta = 0.37
    p_formed = r_old + beta * p_old
    assert np.allclose(p_formed + (r_new - r_old), r_new + beta * p_old, rtol=0, atol=1e-14)


def test_folded_cg_converges_like_textbook():
    """To a residual of 1e-10 both need the same number of iterations."""
    sp, b = _split_problem()
    ref = ow.cg(sp, b, 1e-10, 2000)
    bn = math.sqrt(float(np.vdot(b, b)))
    for k in range(ref["iterations"] - 2, ref["iterations"] + 1):
        x, _, _, _ = folded_cg(sp.apply, b, k)
        rel = np.linalg.norm(b - sp.apply(x)) / bn
        if k < ref["iterations"]:
            assert rel > 1e-10 * 0.5
    assert rel <= 2e-10


def test_noise_part_decomposition():
    """The folded iteration keeps q' = C (nbar W) C p and forms the rest of
    q = (C A C) p from p itself: q = (I - P0) p + q' (P0 the monopole
    projection; Lambda_0 = 0 for the flat monopole prior), p.q' = nbar
    sum(w (C p)^2) (what the z middle pass sums, up to the transform's
    normalisation), and p.q, q.q from p.p without the monopole, p.q', q'.q'
    and the monopole's p(0) q'(0) -- written out on the oracle's real-space
    prior-split system."""
    sp, _ = _split_problem(n=8, nbar=7.0)
    base = sp.base
    rng = np.random.Generator(np.random.PCG64(21))
    p = rng.standard_normal((8,) * 3)
    q = sp.apply(p)
    cp = sp.split(p)
    qn = sp.split(base.nw * cp)
    p_nm = p - p.mean()                       # (I - P0) p
    assert np.allclose(q, p_nm + qn, rtol=0, atol=1e-12 * np.abs(q).max())
    pqn = float(np.vdot(p, qn))
    assert abs(pqn / float(np.sum(base.nw * cp * cp)) - 1.0) < 1e-12
    # in the Fourier basis: the monopole term is the mean's
    m = p.size
    p0q0 = m * p.mean() * qn.mean()           # p(0) q'(0) / M for numpy's unnormalised DFT
    pp = float(np.vdot(p_nm, p_nm))
    pq = pp + pqn
    qq = pp + 2.0 * (pqn - p0q0) + float(np.vdot(qn, qn))
    assert abs(pq / float(np.vdot(p, q)) - 1.0) < 1e-12
    assert abs(qq / float(np.vdot(q, q)) - 1.0) < 1e-12
