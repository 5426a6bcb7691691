"""Rounding sensitivity of fixed-iteration CG (test infrastructure, no GPU).

Two implementations of the same operator round differently, so their k-th
CG iterates differ by an amount that depends on the problem and on k, not on
either implementation being wrong.  This module measures that amount on the
oracle alone: every operator application is multiplied element by element by
(1 + EPS xi), xi standard normal from a seeded generator, and the right-hand
side by (1 + EPS_B xi'), and the perturbed k-th iterate is compared with the
unperturbed one.  EPS = 1e-15 bounds the relative rounding of an FP64 3D FFT
of these sizes (about sqrt(log2 M) 1.1e-16 = 5e-16 at 48^3); EPS_B = 1e-14 is
the agreement of the gridded data with the oracle's (the n^o parity bound is
1e-13 of its maximum, measured 2.5e-14).

SPREADS holds the spreads measured this way (the larger of two seed pairs)
for the workloads and iteration counts of the fixed-iteration GPU tests;
tests/test_oracle_sensitivity.py re-measures them on the CPU.  A GPU bound is
FACTOR times the spread (at least FLOOR).
"""
from __future__ import annotations

import math

import numpy as np

from oracle import wiener as ow

EPS = 1e-15
EPS_B = 1e-14
FACTOR = 5.0
FLOOR = 1e-13

# (workload, form, k) -> relative L2 spread of the k-th iterate
SPREADS = {
    ("pl32", "plain", 50): 3.2e-5,
    ("pl32", "plain", 300): 1.9e-6,
    ("bbks48", "plain", 50): 3.4e-9,
    ("bbks48", "plain", 300): 7.8e-13,
    ("bbks48", "split", 1): 3.9e-15,
    ("bbks48", "split", 20): 9.2e-10,
    ("bbks48", "split", 80): 2.3e-8,
    ("bbks48", "split", 200): 3.4e-14,
}


def bound(workload, form, k):
    """The fixed-iteration parity bound of a GPU test."""
    return max(FACTOR * SPREADS[(workload, form, k)], FLOOR)


class PerturbedSystem:
    """An oracle system whose every application is perturbed by relative
    noise of size eps (seeded)."""

    def __init__(self, base, eps=EPS, seed=0):
        self.base = base
        self.eps = eps
        self.rng = np.random.Generator(np.random.PCG64(seed))

    def apply(self, v):
        a = self.base.apply(v)
        return a * (1.0 + self.eps * self.rng.standard_normal(a.shape))


def perturbed_rhs(b, seed, eps=EPS_B):
    """b times (1 + eps xi), xi standard normal (seeded)."""
    rng = np.random.Generator(np.random.PCG64(1000 + seed))
    return b * (1.0 + eps * rng.standard_normal(np.shape(b)))


def rel_l2(a, b):
    d = np.asarray(a) - b
    return math.sqrt(float(np.vdot(d, d)) / float(np.vdot(b, b)))


def plain_spreads(system, b, ks, seeds=(1, 2), eps=EPS, eps_b=EPS_B):
    """{k: largest relative L2 distance between the oracle's k-th plain CG
    iterate and the k-th iterates of the perturbed runs}, and the
    unperturbed run (its `kept` iterates)."""
    ks = sorted(ks)
    ref = ow.cg(system, b, 0.0, ks[-1], keep=ks)
    worst = {k: 0.0 for k in ks}
    for s in seeds:
        run = ow.cg(PerturbedSystem(system, eps, s), perturbed_rhs(b, s, eps_b), 0.0, ks[-1],
                    keep=ks)
        for k in ks:
            worst[k] = max(worst[k], rel_l2(run["kept"][k], ref["kept"][k]))
    return worst, ref


def split_spreads(system, b, ks, seeds=(1, 2), eps=EPS, eps_b=EPS_B):
    """The same for CG on the prior-split system (C A C) y = C b, compared on
    s = C y."""
    ks = sorted(ks)
    sp = ow.SplitSystem(system)
    cb = sp.split(b)
    ref = ow.cg(sp, cb, 0.0, ks[-1], keep=ks)
    worst = {k: 0.0 for k in ks}
    for s in seeds:
        run = ow.cg(PerturbedSystem(sp, eps, s), sp.split(perturbed_rhs(b, s, eps_b)), 0.0,
                    ks[-1], keep=ks)
        for k in ks:
            worst[k] = max(worst[k], rel_l2(sp.split(run["kept"][k]), sp.split(ref["kept"][k])))
    return worst, ref


def plain_spread(system, b, k, seeds=(1, 2), eps=EPS, eps_b=EPS_B):
    """plain_spreads for one k: (spread, the unperturbed oracle run)."""
    w, ref = plain_spreads(system, b, [k], seeds, eps, eps_b)
    return w[k], ref
