"""Pins of the oracle's fixed-point deposit (Sec. 3.1.2, def:ngrid)."""
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import deposit as od
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "assignment_weights.txt")


def _golden_rows():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line:
                f = line.split()
                rows.append((f[0], int(f[1]), int(f[2]), int(f[3]),
                             [int(v) for v in f[4:]]))
    return rows


@pytest.mark.parametrize("row", _golden_rows())
def test_axis_weights_golden(row):
    scheme, num, den, first_rel, expect = row
    node = 37
    if scheme == "cic":
        U = (node << od.F_BITS) + (num << od.F_BITS) // den
    else:
        U = (node << od.F_BITS) + (num * (1 << od.F_BITS)) // den
    first, w = od.axis_weights(np.array([U]), scheme)
    assert int(first[0]) == node + first_rel
    assert w[0].tolist() == expect


def _textbook_weights(U, scheme):
    """Textbook kernels evaluated exactly (Fractions) at the fixed-point
    position, rounded half up; middle/left weight is the complement."""
    pos = Fraction(U, 1 << od.F_BITS)
    one = 1 << od.Q_BITS

    def rnd(fr):
        return int((fr * one + Fraction(1, 2)) // 1)

    if scheme == "ngp":
        return int((pos + Fraction(1, 2)) // 1), [1]
    if scheme == "cic":
        base = int(pos // 1)
        f = pos - base
        w1 = rnd(f)
        return base, [one - w1, w1]
    nearest = int((pos + Fraction(1, 2)) // 1)
    d = pos - nearest
    wm = rnd((Fraction(1, 2) - d) ** 2 / 2)
    wp = rnd((Fraction(1, 2) + d) ** 2 / 2)
    return nearest - 1, [wm, one - wm - wp, wp]


@pytest.mark.parametrize("scheme", ["ngp", "cic", "tsc"])
def test_axis_weights_match_textbook(scheme):
    rng = np.random.Generator(np.random.PCG64(7))
    U = rng.integers(0, 64 << od.F_BITS, size=400)
    # include exact ties and cell edges
    U = np.concatenate([U, np.array([0, 1, (1 << 23), (1 << 23) - 1, (1 << 24) - 1,
                                     (5 << 24) + (1 << 23), (9 << 24) + (3 << 22)])])
    first, w = od.axis_weights(U, scheme)
    for i, u in enumerate(U.tolist()):
        f_ref, w_ref = _textbook_weights(u, scheme)
        assert int(first[i]) == f_ref
        assert w[i].tolist() == w_ref


def test_tsc_middle_weight_is_textbook_within_one_unit():
    rng = np.random.Generator(np.random.PCG64(8))
    U = rng.integers(0, 64 << od.F_BITS, size=300)
    _, w = od.axis_weights(U, "tsc")
    for i, u in enumerate(U.tolist()):
        pos = Fraction(u, 1 << od.F_BITS)
        d = pos - int((pos + Fraction(1, 2)) // 1)
        mid = (Fraction(3, 4) - d * d) * (1 << od.Q_BITS)
        assert abs(Fraction(int(w[i, 1])) - mid) <= 1


def test_fixed_point_is_one_multiply_and_wrap():
    n_d, box = 64, 500.0
    x = np.array([0.0, 1e-300, 250.0, np.nextafter(500.0, 0.0), 123.456])
    U = od.fixed_point(x, n_d, box)
    c = Fraction(n_d) / Fraction(box)
    for xi, ui in zip(x.tolist(), U.tolist()):
        u = float(xi * (n_d / box))
        if u >= n_d:
            u -= n_d
        assert ui == int(Fraction(u) * (1 << od.F_BITS) // 1)
        assert 0 <= ui < n_d << od.F_BITS
    assert c > 0


@pytest.mark.parametrize("scheme,unit_total", [("ngp", 1), ("cic", 1 << 39),
                                              ("tsc", 1 << 39)])
def test_mass_conservation_exact(scheme, unit_total):
    xyz = synth.uniform_catalogue(5000, 300.0, seed=3)
    g = od.deposit(xyz, 24, 300.0, scheme)
    assert g.dtype == np.int64
    assert int(g.sum()) == 5000 * unit_total
    idx, wt = od.galaxy_stencils(xyz[:50], 24, 300.0, scheme)
    per = wt.reshape(50, -1).sum(axis=1)
    assert np.all(per == unit_total)


def test_ngp_equals_brute_force_count():
    n, box = 16, 200.0
    xyz = synth.uniform_catalogue(3000, box, seed=5)
    g = od.deposit(xyz, n, box, "ngp")
    ref = np.zeros((n, n, n), dtype=np.int64)
    h = box / n
    for x, y, z in xyz.tolist():
        i = int(np.floor(x / h + 0.5)) % n
        j = int(np.floor(y / h + 0.5)) % n
        k = int(np.floor(z / h + 0.5)) % n
        ref[i, j, k] += 1
    assert np.array_equal(g, ref)


@pytest.mark.parametrize("scheme", ["cic", "tsc"])
def test_brute_force_per_galaxy_loop(scheme):
    n, box = 12, 96.0
    xyz = synth.uniform_catalogue(200, box, seed=9)
    g = od.deposit(xyz, n, box, scheme)
    ref = np.zeros((n, n, n), dtype=np.int64)
    for gal in xyz:
        U = [int(Fraction(float(v * (n / box))) * (1 << od.F_BITS) // 1) for v in gal]
        st = [_textbook_weights(u, scheme) for u in U]
        for a, wa in enumerate(st[0][1]):
            for b_, wb in enumerate(st[1][1]):
                for c, wc in enumerate(st[2][1]):
                    ref[(st[0][0] + a) % n, (st[1][0] + b_) % n,
                        (st[2][0] + c) % n] += wa * wb * wc
    assert np.array_equal(g, ref)


@pytest.mark.parametrize("scheme", ["ngp", "cic", "tsc"])
def test_translation_by_whole_cell_rolls_grid(scheme):
    # L = 256, N_d = 32: c = 1/8 exactly; positions on a dyadic lattice are
    # exact, so shifting by H = 8 shifts U by exactly 2^F.
    rng = np.random.Generator(np.random.PCG64(11))
    xyz = rng.integers(0, 256 * 1024 - 8 * 1024, size=(400, 3)).astype(np.float64) / 1024
    g0 = od.deposit(xyz, 32, 256.0, scheme)
    g1 = od.deposit(xyz + np.array([8.0, 0.0, 16.0]), 32, 256.0, scheme)
    assert np.array_equal(np.roll(g0, (1, 0, 2), axis=(0, 1, 2)), g1)


def test_order_independence():
    xyz = synth.uniform_catalogue(2000, 100.0, seed=12)
    perm = np.random.Generator(np.random.PCG64(1)).permutation(len(xyz))
    for scheme in ("ngp", "cic", "tsc"):
        assert np.array_equal(od.deposit(xyz, 16, 100.0, scheme),
                              od.deposit(xyz[perm], 16, 100.0, scheme))


def test_deposit_at_matches_full_grid():
    xyz = synth.uniform_catalogue(4000, 100.0, seed=13)
    g = od.deposit(xyz, 20, 100.0, "tsc")
    rng = np.random.Generator(np.random.PCG64(2))
    nodes = rng.integers(0, 20, size=(40, 3))
    got = od.deposit_at(xyz, 20, 100.0, "tsc", nodes)
    assert np.array_equal(got, g[nodes[:, 0], nodes[:, 1], nodes[:, 2]])


def test_wrap_at_upper_edge():
    # x just below L can round to u = N_d exactly; it must land on node 0.
    box = 0.1
    x = np.nextafter(box, 0.0)
    n_d = 3
    u = x * (n_d / box)
    U = od.fixed_point(np.array([x]), n_d, box)
    assert 0 <= int(U[0]) < n_d << od.F_BITS
    if u >= n_d:
        assert int(U[0]) == 0
