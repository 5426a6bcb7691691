"""Fixed-point mass assignment (oracle; test infrastructure only).

Sec. 3.1.2 (def:ngrid) defines gridding as a convolution of the point-source
galaxy field with an assignment kernel, followed by sampling on a Dirac comb at
integer multiples of the spacing H; it names the NGP, CIC and TSC kernels and
uses TSC on a grid of twice the target resolution.

Readings taken here (the paper gives no discretisation details):

* nodes sit at x_n = n H, n in [0, N_d), periodic (the comb of def:ngrid);
* coordinates go to fixed point: u = x * (N_d / L) (one FP64 multiply), wrapped
  once if u >= N_d, then U = floor(u * 2^F) with F = 24 (exact);
* per-axis weights are integers in units of 2^-Q, Q = 13, rounded half up, and
  the middle TSC / left CIC weight is the complement, so the weights of one
  galaxy sum to exactly 2^Q per axis and 2^(3Q) in 3D;
* NGP deposits plain counts (weight 1, unit 1); CIC/TSC deposit products
  Wx Wy Wz in units of 2^-39;
* the accumulation is integer, hence exact and independent of galaxy order.
"""
from __future__ import annotations

import numpy as np

F_BITS = 24
Q_BITS = 13
HALF = 1 << (F_BITS - 1)
ONE_Q = 1 << Q_BITS


def scheme_unit(scheme):
    """Real value of one integer deposit unit."""
    return 1.0 if scheme == "ngp" else 2.0 ** (-3 * Q_BITS)


def fixed_point(xyz, n_d, box):
    """u = x * (N_d/L), wrap once at N_d, U = floor(u * 2^F) as int64."""
    xyz = np.asarray(xyz, dtype=np.float64)
    c = np.float64(n_d) / np.float64(box)
    u = xyz * c
    u = np.where(u >= n_d, u - n_d, u)
    return np.floor(u * float(1 << F_BITS)).astype(np.int64)


def axis_weights(U, scheme):
    """Per-axis stencil for fixed-point coordinates U (int64 array).

    Returns (first_node, weights) where weights has shape U.shape + (S,),
    S = 1, 2, 3 for NGP, CIC, TSC, and node j of the stencil is
    first_node + j (before the periodic wrap).
    """
    U = np.asarray(U, dtype=np.int64)
    if scheme == "ngp":
        node = (U + HALF) >> F_BITS
        return node, np.ones(U.shape + (1,), dtype=np.int64)
    if scheme == "cic":
        node = U >> F_BITS
        frac = U & ((1 << F_BITS) - 1)
        w1 = (frac + (1 << (F_BITS - Q_BITS - 1))) >> (F_BITS - Q_BITS)
        w0 = ONE_Q - w1
        return node, np.stack([w0, w1], axis=-1)
    if scheme == "tsc":
        node = (U + HALF) >> F_BITS
        d = U - (node << F_BITS)             # in [-2^(F-1), 2^(F-1))
        sh = 2 * F_BITS + 1 - Q_BITS         # 36
        rnd = 1 << (sh - 1)
        wm = ((HALF - d) ** 2 + rnd) >> sh
        wp = ((HALF + d) ** 2 + rnd) >> sh
        w0 = ONE_Q - wm - wp
        return node - 1, np.stack([wm, w0, wp], axis=-1)
    raise ValueError(f"unknown scheme {scheme!r}")


def galaxy_stencils(xyz, n_d, box, scheme):
    """Flat node indices and int64 weights of every (galaxy, stencil node)."""
    U = fixed_point(xyz, n_d, box)
    first, w = axis_weights(U, scheme)        # (n,3), (n,3,S)
    s = w.shape[-1]
    offs = np.arange(s, dtype=np.int64)
    ix = (first[:, 0, None] + offs) % n_d     # (n,S)
    iy = (first[:, 1, None] + offs) % n_d
    iz = (first[:, 2, None] + offs) % n_d
    flat = (ix[:, :, None, None] * n_d + iy[:, None, :, None]) * n_d + iz[:, None, None, :]
    wt = w[:, 0, :, None, None] * w[:, 1, None, :, None] * w[:, 2, None, None, :]
    return flat.reshape(-1), wt.reshape(-1)


def deposit(xyz, n_d, box, scheme, chunk=1 << 18):
    """Integer grid G[n_d,n_d,n_d] (int64): the sum over galaxies of their
    stencil weights (def:ngrid sampled on the comb)."""
    grid = np.zeros(n_d ** 3, dtype=np.int64)
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    for lo in range(0, xyz.shape[0], chunk):
        idx, wt = galaxy_stencils(xyz[lo:lo + chunk], n_d, box, scheme)
        np.add.at(grid, idx, wt)
    return grid.reshape(n_d, n_d, n_d)


def deposit_at(xyz, n_d, box, scheme, nodes, chunk=1 << 18):
    """G at the listed nodes ((k,3) int array), evaluated one node at a time
    from the galaxies whose stencil covers it -- usable at sizes where the
    whole grid is not formed."""
    nodes = np.asarray(nodes, dtype=np.int64).reshape(-1, 3)
    flat_nodes = (nodes[:, 0] * n_d + nodes[:, 1]) * n_d + nodes[:, 2]
    out = np.zeros(len(flat_nodes), dtype=np.int64)
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    order = np.argsort(flat_nodes)
    sorted_nodes = flat_nodes[order]
    for lo in range(0, xyz.shape[0], chunk):
        idx, wt = galaxy_stencils(xyz[lo:lo + chunk], n_d, box, scheme)
        pos = np.searchsorted(sorted_nodes, idx)
        pos = np.minimum(pos, len(sorted_nodes) - 1)
        hit = sorted_nodes[pos] == idx
        acc = np.zeros(len(sorted_nodes), dtype=np.int64)
        np.add.at(acc, pos[hit], wt[hit])
        out[order] += acc
    return out
