"""Writes an oracle reference solution of a named workload (no GPU involved).

The reference is the oracle's plain CG (FP64, scipy's multi-threaded FFT)
run to a relative residual of 1e-12 on the workload's synthetic inputs, from
the oracle's own deposit and low-pass.  It is stored as float32 (the
comparison it serves is at the 1e-6 level) with a JSON sidecar.

    python tests/golden/make_reference.py bbks512 OUTDIR [--workers 8]

With --sample-from FULL.npy it instead reads such a stored reference and
writes every --stride-th cell along each axis (cells [::s, ::s, ::s]) to
OUTDIR/<workload>_n<n>_x_s<s>.npy: the sampled outputs a full-size GPU test
compares against.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import supersample as oss  # noqa: E402
from oracle import wiener as ow  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload")
    ap.add_argument("outdir")
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--tol", type=float, default=1e-12)
    ap.add_argument("--workers", type=int, default=os.cpu_count())
    ap.add_argument("--sample-from", default=None)
    ap.add_argument("--stride", type=int, default=8)
    a = ap.parse_args()
    os.makedirs(a.outdir, exist_ok=True)
    wl = synth.workload(a.workload, n=a.n)
    if a.sample_from:
        full = np.load(a.sample_from, mmap_mode="r")
        st = a.stride
        sample = np.ascontiguousarray(full[::st, ::st, ::st], dtype=np.float32)
        out = os.path.join(a.outdir, f"{wl.name}_n{wl.n}_x_s{st}.npy")
        np.save(out, sample)
        print("wrote", out, sample.shape, flush=True)
        return
    t0 = time.time()
    ptab = wl.ptab()
    w = wl.mask()
    cat = wl.catalogue(ptab, w)
    print(f"inputs {wl.name} n={wl.n} ngal={len(cat.xyz)} ({time.time() - t0:.0f} s)", flush=True)
    n_obs, grid = oss.observed_counts(cat.xyz, wl.n, wl.box, wl.scheme, wl.supersample)
    del grid
    nbar = ow.mean_density(len(cat.xyz), w)
    b = ow.data_vector(n_obs, w, nbar)
    print(f"data vector ({time.time() - t0:.0f} s) nbar={nbar:.6g}", flush=True)
    system = ow.System(wl.n, wl.box, w, ptab, nbar, workers=a.workers)
    hist = []
    res = ow.cg(system, b, a.tol, 100000, record=hist)
    print(f"cg {res['iterations']} its rel_res={res['rel_res']:.3e} "
          f"true={res['rel_res_true']:.3e} ({time.time() - t0:.0f} s)", flush=True)
    stem = os.path.join(a.outdir, f"{wl.name}_n{wl.n}")
    np.save(stem + "_x.npy", res["x"].astype(np.float32))
    lo, hi = ow.lanczos_extremes(res["alphas"], res["betas"])
    meta = dict(workload=wl.name, n=wl.n, box=wl.box, seed=wl.seed, n_gal=int(len(cat.xyz)),
                nbar=nbar, iterations=res["iterations"], rel_res=res["rel_res"],
                rel_res_true=res["rel_res_true"], tol=a.tol, ritz_min=lo, ritz_max=hi,
                residual_history=hist[::10], x_norm=float(np.linalg.norm(res["x"])))
    with open(stem + "_meta.json", "w") as fh:
        json.dump(meta, fh)
    print("wrote", stem, flush=True)


if __name__ == "__main__":
    main()
