"""Writes oracle fixed-iteration and converged references of a named workload
at sampled cells (no GPU involved; calls only oracle/ and synth/ plus the
noise wrapper of tests/sensitivity.py).

For the workload's synthetic inputs it runs the oracle's whole path (integer
deposit, low-pass, data vector) and then, on the plain FP64 system:

* exactly k CG iterations for every k of --ks, and the spread of those
  iterates under the noise model of tests/sensitivity.py (1e-15 relative
  noise in every transform stage, 1e-15 of the largest value on the data;
  two seeds): the
  rounding sensitivity the fixed-k GPU bounds are derived from;
* CG to the relative residual --tol (the workload's own stopping rule): the
  oracle's result at that stop;
* a tight reference A^-1 b (the oracle's PCG to 1e-13).

Every vector is stored at cells [::s, ::s, ::s] (--stride s) in float64 in
OUTDIR/<workload>_n<n>_cg.npz, with full-grid norms, iteration counts and
residuals in OUTDIR/<workload>_n<n>_cg.json.

    python tests/golden/make_fixed_k.py bbks256 tests/golden --ks 50,300 --tol 1e-6

With --spreads-only it re-measures the spreads alone and rewrites them into
an existing JSON file (the stored vectors do not depend on the noise model).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import synth  # noqa: E402
from oracle import supersample as oss  # noqa: E402
from oracle import wiener as ow  # noqa: E402
import sensitivity  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload")
    ap.add_argument("outdir")
    ap.add_argument("--ks", default="50,300")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--stride", type=int, default=8)
    ap.add_argument("--workers", type=int, default=os.cpu_count())
    ap.add_argument("--spreads-only", action="store_true")
    a = ap.parse_args()
    t0 = time.time()

    def log(msg):
        print(f"[{time.time() - t0:7.0f} s] {msg}", flush=True)

    wl = synth.workload(a.workload)
    ptab = wl.ptab()
    w = wl.mask()
    cat = wl.catalogue(ptab, w)
    log(f"inputs {wl.name} n={wl.n} ngal={len(cat.xyz)}")
    n_obs, grid = oss.observed_counts(cat.xyz, wl.n, wl.box, wl.scheme, wl.supersample)
    mass = int(grid.sum())
    del grid
    nbar = ow.mean_density(len(cat.xyz), w)
    b = ow.data_vector(n_obs, w, nbar)
    log(f"data vector nbar={nbar:.6g}")
    system = ow.System(wl.n, wl.box, w, ptab, nbar, workers=a.workers)
    st = a.stride
    arrays = {"n_obs": n_obs[::st, ::st, ::st].copy(), "b": b[::st, ::st, ::st].copy()}
    meta = dict(workload=wl.name, n=wl.n, box=wl.box, seed=wl.seed, n_gal=int(len(cat.xyz)),
                scheme=wl.scheme, supersample=wl.supersample, stride=st, nbar=nbar,
                deposit_total=mass, b_norm=float(np.linalg.norm(b)), fixed_k={})
    ks = sorted(int(s) for s in a.ks.split(","))
    spreads, _ = sensitivity.plain_spreads(system, b, ks)
    stem = os.path.join(a.outdir, f"{wl.name}_n{wl.n}_cg")
    if a.spreads_only:
        with open(stem + ".json") as fh:
            old = json.load(fh)
        for k in ks:
            old["fixed_k"][str(k)]["spread"] = spreads[k]
            log(f"k={k}: spread {spreads[k]:.3e}")
        with open(stem + ".json", "w") as fh:
            json.dump(old, fh, indent=1)
        log(f"rewrote the spreads in {stem}.json")
        return
    for k in ks:
        ref = ow.cg(system, b, 0.0, k)
        arrays[f"x_k{k}"] = ref["x"][::st, ::st, ::st].copy()
        meta["fixed_k"][str(k)] = dict(rel_res=ref["rel_res"], rel_res_true=ref["rel_res_true"],
                                       x_norm=float(np.linalg.norm(ref["x"])), spread=spreads[k])
        log(f"k={k}: rel_res {ref['rel_res']:.6e} spread {spreads[k]:.3e}")
    res = ow.cg(system, b, a.tol, 100000)
    arrays["x_tol"] = res["x"][::st, ::st, ::st].copy()
    meta["stop"] = dict(tol=a.tol, iterations=res["iterations"], rel_res=res["rel_res"],
                        rel_res_true=res["rel_res_true"], x_norm=float(np.linalg.norm(res["x"])))
    log(f"cg to {a.tol:g}: {res['iterations']} iterations, true {res['rel_res_true']:.3e}")
    ref = ow.reference_solution(system, b, tol=1e-13, max_iter=50000)
    xr = ref["x"]
    rt = b - system.apply(xr)
    arrays["x_ref"] = xr[::st, ::st, ::st].copy()
    meta["reference"] = dict(method="pcg", tol=1e-13, iterations=ref["iterations"],
                             rel_res_true=float(np.linalg.norm(rt) / np.linalg.norm(b)),
                             x_norm=float(np.linalg.norm(xr)),
                             stop_error=ow.error_l2(res["x"], xr))
    log(f"reference: {ref['iterations']} PCG iterations, stop error {meta['reference']['stop_error']:.3e}")
    np.savez(stem + ".npz", **arrays)
    with open(stem + ".json", "w") as fh:
        json.dump(meta, fh, indent=1)
    log(f"wrote {stem}.npz / .json")


if __name__ == "__main__":
    main()
