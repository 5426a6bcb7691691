"""Rounding sensitivity of fixed-iteration CG (test infrastructure, no GPU).

Two implementations of the same operator round differently, so their k-th
CG iterates differ by an amount that depends on the problem and on k, not on
either implementation being wrong.  This module measures that amount on the
oracle alone, with every operator application rounded like an FFT pipeline:
white noise of EPS times the root mean square of each transformed field is
added to it -- to the forward spectrum before the Fourier diagonal multiplies
it (so the forward transform's error is scaled by Lambda, or by the split
factor, as in any implementation) and to the result of each inverse
transform -- and the right-hand side, on its observed cells, EPS_B times its
largest magnitude.  A 3D FFT's rounding is of that form, about
sqrt(log2 M) 1.1e-16 of the field's norm spread over every element (5e-16 at
256^3), and EPS = 1e-15 bounds it at the sizes tested.  The gridded data come
out of the FFT low-pass, so their rounding is absolute too, of the order of
the largest count: n^o agrees with the oracle's to 4e-16 of its maximum at
256^3, and EPS_B = 1e-15 bounds that.  For the lognormal fields of these
workloads the largest |b| is ~2000 times its root mean square, which makes
the data's rounding, not the operator's, the larger source at small k.  The
perturbed k-th iterate is compared with the unperturbed one.

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
EPS_B = 1e-15
FACTOR = 5.0
FLOOR = 1e-13

# (workload, form, k) -> relative L2 spread of the k-th iterate
SPREADS = {
    ("pl32", "plain", 50): 3.1e-5,
    ("pl32", "plain", 300): 2.0e-6,
    ("bbks48", "plain", 50): 6.9e-10,
    ("bbks48", "plain", 300): 2.6e-13,
    ("bbks48", "split", 1): 8.7e-15,
    ("bbks48", "split", 20): 2.0e-9,
    ("bbks48", "split", 80): 2.4e-8,
    ("bbks48", "split", 200): 4.6e-14,
}


def bound(workload, form, k):
    """The fixed-iteration parity bound of a GPU test."""
    return max(FACTOR * SPREADS[(workload, form, k)], FLOOR)


def _rms(a):
    return math.sqrt(float(np.vdot(a, a).real) / a.size)


class PerturbedSystem:
    """An oracle plain system (oracle.wiener.System) whose every application
    rounds like an FFT pipeline: white noise of eps times the root mean square
    of the forward spectrum is added before the Fourier diagonal multiplies
    it (so, as in any implementation, the forward transform's error is
    scaled by Lambda), and of eps times that of the result after the inverse
    transform (seeded)."""

    def __init__(self, base, eps=EPS, seed=0):
        self.base = base
        self.eps = eps
        self.rng = np.random.Generator(np.random.PCG64(seed))

    def _noise(self, a):
        if np.iscomplexobj(a):
            z = self.rng.standard_normal(a.shape) + 1j * self.rng.standard_normal(a.shape)
            return (self.eps * _rms(a) / math.sqrt(2.0)) * z
        return (self.eps * _rms(a)) * self.rng.standard_normal(a.shape)

    def apply(self, v):
        b = self.base
        vk = b._rfft(v)
        vk = vk + self._noise(vk)
        out = b._irfft(b.lam * vk)
        return out + self._noise(out) + b.nw * v


class PerturbedSplit:
    """The prior-split system (C A C) of an oracle system with the same
    rounding model: the forward spectra of its real-space stage get noise of
    eps times their size before the split factor multiplies them, the real
    field after the inverse transform likewise (seeded)."""

    def __init__(self, sp, eps=EPS, seed=0):
        self.sp = sp
        self.pert = PerturbedSystem(sp.base, eps, seed)

    def apply(self, y):
        sp, pb = self.sp, self.pert
        b = sp.base
        u = b._irfft(sp.c * b._rfft(y))              # C y
        u = u + pb._noise(u)
        g = b.nw * u                                  # the noise term of A on C y
        gk = b._rfft(g)
        gk = gk + pb._noise(gk)
        out = b._irfft(sp.c * gk)                     # C n w C y
        out = out + pb._noise(out)
        # the prior part of C A C is the identity off the monopole
        yk = b._rfft(y)
        yk[0, 0, 0] = 0.0
        return out + b._irfft(yk)


def perturbed_rhs(b, seed, eps=EPS_B):
    """b plus white noise of eps times its largest magnitude on the cells where
    it is not zero (seeded): the rounding of a gridded field produced by FFTs
    is absolute, of the order of the largest value."""
    b = np.asarray(b, dtype=np.float64)
    rng = np.random.Generator(np.random.PCG64(1000 + seed))
    noise = (eps * float(np.abs(b).max())) * rng.standard_normal(b.shape)
    return b + np.where(b != 0.0, noise, 0.0)


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
        run = ow.cg(PerturbedSplit(sp, eps, s), sp.split(perturbed_rhs(b, s, eps_b)), 0.0,
                    ks[-1], keep=ks)
        for k in ks:
            worst[k] = max(worst[k], rel_l2(sp.split(run["kept"][k]), sp.split(ref["kept"][k])))
    return worst, ref


def plain_spread(system, b, k, seeds=(1, 2), eps=EPS, eps_b=EPS_B):
    """plain_spreads for one k: (spread, the unperturbed oracle run)."""
    w, ref = plain_spreads(system, b, [k], seeds, eps, eps_b)
    return w[k], ref
