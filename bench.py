"""Throughput of the Wiener reconstruction on one MI355X.

One step = the whole hot path on one synthetic catalogue with every input
already in HBM: copy in the galaxies, fixed-point TSC deposit on the 1024^3
grid, ideal low-pass to 512^3, data vector, and the mixed-precision CG solve
of the Wiener system (by default on the prior-split system; FP32 operator and
FFTs, FP64 dots, FP64 residual recomputation with reliable updates) to the
refinement tolerance.

Prints one JSON line: solves/s, the roofline figure of the dominant kernel
(HIP events around its launches during the timed steps), the error against
the oracle's stored reference solution, the FP64 and plain-CG comparisons, the
oracle timed on the host cores, the post-solve functions, and (each can be
switched off with 0) a 16-RHS batch at 256^3, a serving stream, 200
signal-dependent-noise jackknife solves at 128^3 and the deposit of 2e6
galaxies from spread out to piled on one point.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np
import xxhash

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, 8 TB/s
# Outer (FP64) residual tolerance of the refinement per preconditioning,
# chosen so that the error against the FP64 solution stays below 1e-6 with a
# margin.  Plain CG stops on ||b - A s|| / ||b||, whose error is ~200x the
# residual on the 512^3 workload (2e-9 -> 4.5e-7); the prior-split CG stops on
# ||C (b - A s)|| / ||C b||, whose error is about the residual (3e-7 -> 2.2e-7).
TOLERANCES = {"none": 2e-9, "prior": 3e-7}
DEFAULT_TOL = TOLERANCES["none"]
KERNEL_SOURCES = ["paper_0906_3978_amd/csrc/fftpass.hip", "paper_0906_3978_amd/csrc/kernels.hip",
                  "paper_0906_3978_amd/csrc/fft.h",
                  "paper_0906_3978_amd/csrc/common.h"]


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_inputs(name, n_override=None):
    import synth
    wl = synth.workload(name, n=n_override)
    t = time.perf_counter()
    ptab = wl.ptab()
    w = wl.mask()
    cat = wl.catalogue(ptab, w)
    log(f"[bench] inputs {wl.name} n={wl.n} ngal={len(cat.xyz)} sigma_G^2={cat.sigma_g2:.2f} "
        f"({time.perf_counter() - t:.1f} s)")
    return wl, ptab, w, cat


class _IterationClock(list):
    """Passed as the oracle CG's `record` list: stamps the time of every
    iteration's end, so that the span between two stamps is one iteration."""

    def append(self, value):
        super().append(time.perf_counter())


def cpu_baseline(wl, ptab, w, xyz, iters_fp64, precond="prior", cg_iters=20):
    """The oracle timed on the host, phase by phase, on the workload's own
    catalogue: its integer deposit, its low-pass (scipy's FFT on the host's
    threads, at most 16), the data vector, and `cg_iters` FP64 CG iterations
    (prior-split CG for precond="prior": the oracle forms C A C as three FFT
    pairs per iteration, where the library needs one), whose median
    iteration time is extrapolated to the `iters_fp64` iterations of an FP64
    solve of the same system.  Returns the baseline and its per-phase times."""
    from oracle import deposit as od
    from oracle import supersample as oss
    from oracle import wiener as ow
    workers = min(16, os.cpu_count() or 1)
    t = time.perf_counter()
    grid = od.deposit(xyz, wl.supersample * wl.n, wl.box, wl.scheme)
    t_dep = time.perf_counter() - t
    t = time.perf_counter()
    g = grid.astype(np.float64) * od.scheme_unit(wl.scheme)
    del grid
    nobs = oss.lowpass_decimate(g, wl.n, workers) if wl.supersample == 2 else g
    del g
    t_lp = time.perf_counter() - t
    t = time.perf_counter()
    nbar = ow.mean_density(len(xyz), w)
    b = ow.data_vector(nobs, w, nbar)
    t_rhs = time.perf_counter() - t
    system = ow.System(wl.n, wl.box, w, ptab, nbar, workers=workers)
    solve = ow.split_cg if precond == "prior" else ow.cg
    clock = _IterationClock()
    t = time.perf_counter()
    solve(system, b, 0.0, cg_iters, record=clock)
    t_cg = time.perf_counter() - t
    spans = np.diff(np.asarray(clock))
    per_it = float(np.median(spans))
    total = t_dep + t_lp + t_rhs + per_it * iters_fp64
    name = "prior-split CG (three FFT pairs per iteration)" if precond == "prior" else "plain CG"
    return {"value": 1.0 / total, "unit": "solves/s", "cores": workers, "kind": "oracle",
            "sample": (f"the oracle on the {wl.n}^3 workload: deposit {t_dep:.2f} s, low-pass "
                       f"{t_lp:.2f} s, data vector {t_rhs:.2f} s, {cg_iters} FP64 {name} "
                       f"iterations ({t_cg:.1f} s, median {per_it:.3f} s each) extrapolated to "
                       f"the {iters_fp64} iterations of the FP64 solve"),
            "phases_s": {"deposit": round(t_dep, 3), "lowpass": round(t_lp, 3),
                         "data_vector": round(t_rhs, 3), "cg_iteration": round(per_it, 4),
                         "cg_iterations_timed": cg_iters, "cg_iterations_extrapolated": iters_fp64},
            "extrapolated": True, "host": host_cpu()}


def _iteration_roofline(prof, keys, n):
    """Per-iteration time, algorithmic bytes and HBM fraction from the live
    profiler's classes of one CG iteration."""
    if not all(k in prof and prof[k]["launches"] for k in keys):
        return None
    it_ms = sum(prof[k]["ms"] / prof[k]["launches"] for k in keys)
    it_b = sum(prof[k]["bytes"] / prof[k]["launches"] for k in keys)
    ach = it_b / (it_ms * 1e-3) / 1e9
    return {"ms": round(it_ms, 4), "bytes": it_b, "achieved_gbs": round(ach, 1),
            "frac": round(ach / HBM_PEAK_GBS, 4), "bytes_per_cell": round(it_b / n ** 3, 2)}


PLAIN_F64 = ["zfwd_f64", "yfwd_f64", "xlam_f64", "yinv_f64", "zinv_f64", "update_f64"]
PLAIN_F32 = ["zfwd_f32", "yfwd_f32", "xlam_f32", "yinv_f32", "zinv_f32", "update_f32"]
# the FP32 prior-split iteration applies r -= alpha q in its first pass (no
# update kernel)
SPLIT_F32 = ["sxinv_f32", "yinv_f32", "szw_f32", "yfwd_f32", "sxfwd_f32"]


def _dominant(prof, keys):
    d = max(keys, key=lambda k: prof[k]["ms"])
    v = prof[d]
    avg = v["ms"] * 1e-3 / v["launches"]
    ach = v["bytes"] / v["launches"] / avg / 1e9
    return {"kernel": d, "avg_launch_us": round(avg * 1e6, 2), "achieved_gbs": round(ach, 1),
            "frac": round(ach / HBM_PEAK_GBS, 4)}


def fp64_config_run(name, reps=3, cpu_full=False):
    """A plain FP64 configuration (pl32: 32^3 power law, NGP, residual 1e-10;
    bbks256: 256^3 BBKS, CIC 2x supersampled, residual 1e-6) on its synthetic
    catalogue already in HBM: gridding plus the FP64 CG solve, median of
    `reps`, with the FP64 iteration's roofline; the oracle beside it (full
    solves, median of 3, when cpu_full, else phases with 20 CG iterations
    extrapolated)."""
    import torch
    import synth
    import paper_0906_3978_amd as wf
    from oracle import wiener as ow
    wl = synth.workload(name)
    tol = 1e-10 if name == "pl32" else 1e-6
    ptab = wl.ptab()
    w = wl.mask()
    cat = wl.catalogue(ptab, w)
    dev = torch.device("cuda:0")
    ctx = wf.Context(0)
    ctx.set_grid(wl.n, wl.box)
    ctx.set_mask(torch.from_numpy(w).to(dev))
    ctx.set_power(torch.from_numpy(ptab).to(dev))
    xyz = torch.from_numpy(cat.xyz).to(dev)
    out = torch.empty((wl.n,) * 3, dtype=torch.float64, device=dev)

    def one():
        ctx.set_galaxies(xyz)
        ctx.deposit(wl.scheme, wl.supersample)
        return ctx.solve(out=out, precision="fp64", tol=tol, max_iter=100000)[1]
    one()
    torch.cuda.synchronize()
    ts, info = [], None
    for _ in range(reps):
        t = time.perf_counter()
        info = one()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
    # the roofline from a separate run with the live profiler on (its events
    # around every launch would slow the timed runs of small grids)
    ctx.profile_enable(True)
    one()
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    ctx.close()
    t_gpu = float(np.median(ts))
    res = {"workload": f"{name}: {wl.n}^3 / {wl.box:.0f} Mpc, {wl.spectrum}, "
                       f"{wl.scheme.upper()} s={wl.supersample}, {len(cat.xyz)} galaxies, "
                       f"plain FP64 CG to {tol:g}",
           "solves_per_s": round(1.0 / t_gpu, 3), "solve_s_median": round(t_gpu, 5),
           "iters": info.iters_total, "rel_res_true": info.rel_res_true,
           "roofline_iteration_fp64": _iteration_roofline(prof, PLAIN_F64, wl.n),
           "dominant_fp64_kernel": _dominant(prof, PLAIN_F64)}
    if cpu_full:
        tc = []
        for _ in range(3):
            t = time.perf_counter()
            r = ow.reconstruct(cat.xyz, wl.n, wl.box, w, ptab, wl.scheme, wl.supersample, tol,
                               100000)
            tc.append(time.perf_counter() - t)
        res["cpu_oracle"] = {"value": round(1.0 / float(np.median(tc)), 4), "unit": "solves/s",
                             "cores": 1, "kind": "oracle",
                             "sample": f"full oracle solves (deposit, data vector, {r['iterations']} "
                                       f"CG iterations), median of 3: "
                                       f"{', '.join(f'{x:.2f}' for x in tc)} s"}
    else:
        res["cpu_oracle"] = cpu_baseline(wl, ptab, w, cat.xyz, info.iters_total, "none")
    res["speedup_vs_cpu_oracle"] = round(res["solves_per_s"] / res["cpu_oracle"]["value"], 1)
    log(f"[{name}] {res}")
    return res


def host_cpu():
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count()}


def _pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = min(len(xs), max(1, math.ceil(q * len(xs))))
    return xs[k - 1]


def serve(n_req, tol, precond="prior", seed=5000, per_grid=6, warmup=20, outstanding=48,
          streams=4):
    """Serving: a stream of reconstruction requests through the
    continuous-batching server.

    Requests are drawn with replacement from a pool of `per_grid` distinct
    request templates per grid size (synth.serving_request: grids 64..384,
    random caps, radial scales, spectrum amplitudes and catalogue sizes), so
    that every result can be checked against the same template served alone.
      A. isolated: every template alone (one at a time) -- reference results
         and the isolated service time; capacity = 1 / mean service time of
         the stream's mix;
      B. Poisson arrivals at 0.7 x capacity: `warmup` requests, then `n_req`
         measured ones; latency (submit -> result on the host) p50 / p99
         overall and per grid size, served solves/s;
      C. saturated: the same `n_req` requests kept `outstanding` at a time
         (closed loop), solves/s and the batched solves formed.
    Every result of B and C must equal its template's result of A bit for bit."""
    import synth
    import paper_0906_3978_amd as wf
    grids = (64, 128, 256, 384)
    t = time.perf_counter()
    templ = []
    counts = {g: 0 for g in grids}
    i = 0
    while min(counts.values()) < per_grid:
        wl = synth.serving_request(i, base_seed=seed + 1)
        i += 1
        if counts[wl.n] >= per_grid:
            continue
        counts[wl.n] += 1
        ptab = wl.ptab()
        w = wl.mask()
        templ.append((wl, w, ptab, wl.catalogue(ptab, w).xyz))
    log(f"[serve] {len(templ)} request templates ({time.perf_counter() - t:.1f} s)")
    budget = 96 << 30
    kw = dict(precision="mixed", tol=tol, max_iter=100000, precond=precond)

    def submit(srv, r):
        wl, w, ptab, xyz = r
        return srv.submit(wl.n, wl.box, w, ptab, xyz, wl.scheme, wl.supersample, **kw)

    def digest(x):
        # bit-for-bit identity of results (xxh3: the host keeps up with the GPU)
        return xxhash.xxh3_128_hexdigest(np.ascontiguousarray(x).view(np.uint8))

    # A: isolated
    alone, service = [], []
    with wf.Server(0, hbm_budget=budget, max_active=1) as srv:
        for r in templ:
            t0 = time.perf_counter()
            x, info = srv.wait(submit(srv, r), r[0].n, timeout=600)
            service.append(time.perf_counter() - t0)
            alone.append(digest(x))
    rng = np.random.Generator(np.random.PCG64(seed))
    pick = rng.integers(0, len(templ), size=warmup + n_req)
    cap = 1.0 / float(np.mean([service[k] for k in pick[warmup:]]))
    rate = 0.7 * cap
    gaps = rng.exponential(1.0 / rate, size=len(pick))

    def collect(srv, tickets, ks):
        out = []
        for tk, k in zip(tickets, ks):
            x, info = srv.wait(tk, templ[k][0].n, timeout=600)
            out.append((k, digest(x), info))
        return out

    # B: Poisson arrivals.  Completion times are submit time + the server's
    # latency, so the host's own work on the results (fetch, digest) stays out
    # of the served rate.
    with wf.Server(0, hbm_budget=budget, max_active=streams) as srv:
        tickets, t_sub = [], []
        t0 = time.perf_counter()
        next_t = 0.0
        for j, (k, g) in enumerate(zip(pick, gaps)):
            next_t += g
            while time.perf_counter() - t0 < next_t:
                time.sleep(0.0002)
            t_sub.append(time.perf_counter() - t0)
            tickets.append(submit(srv, templ[k]))
            if (j + 1) % 100 == 0:
                log(f"[serve] Poisson: {j + 1} of {len(pick)} submitted")
        res_b = collect(srv, tickets, pick)
        span_b = time.perf_counter() - t0
        st_b = srv.stats()
    meas = res_b[warmup:]
    t_first = t_sub[warmup]
    t_last_b = max(t_sub[j] + res_b[j][2].latency_ms * 1e-3 for j in range(warmup, len(res_b)))
    lat = [info.latency_ms for _, _, info in meas]
    per_grid_lat = {}
    for g in grids:
        lg = [info.latency_ms for k, _, info in meas if templ[k][0].n == g]
        if lg:
            per_grid_lat[str(g)] = {"requests": len(lg), "p50_ms": round(_pct(lg, 0.5), 2),
                                    "p99_ms": round(_pct(lg, 0.99), 2)}
    # C: saturated, closed loop
    import collections
    with wf.Server(0, hbm_budget=budget, max_active=streams) as srv:
        inflight = collections.deque()
        res_c, t_sub_c = [], []
        t0 = time.perf_counter()
        for j, k in enumerate(pick[warmup:]):
            if len(inflight) >= outstanding:
                tk, kk = inflight.popleft()
                res_c += collect(srv, [tk], [kk])
            t_sub_c.append(time.perf_counter() - t0)
            inflight.append((submit(srv, templ[k]), k))
            if (j + 1) % 100 == 0:
                log(f"[serve] saturated: {j + 1} of {n_req} submitted")
        while inflight:
            tk, kk = inflight.popleft()
            res_c += collect(srv, [tk], [kk])
        span_c = max(t_sub_c[j] + res_c[j][2].latency_ms * 1e-3 for j in range(len(res_c)))
        st_c = srv.stats()
    same = all(h == alone[k] for k, h, _ in res_b + res_c)
    errs = [info.last_change for _, _, info in res_b + res_c]
    res = {"requests": n_req, "warmup": warmup, "templates": len(templ), "grids": list(grids),
           "streams": streams,
           "isolated_service_ms_per_grid": {str(g): round(1e3 * float(np.mean(
               [service[j] for j in range(len(templ)) if templ[j][0].n == g])), 2) for g in grids},
           "isolated_solves_per_s": round(cap, 4), "arrival_rate_per_s": round(rate, 4),
           "realized_arrival_per_s": round(float((len(t_sub) - 1 - warmup) /
                                                 max(t_sub[-1] - t_sub[warmup], 1e-9)), 4),
           "served_solves_per_s": round(float(len(meas) / max(t_last_b - t_first, 1e-9)), 4),
           "p50_ms": round(_pct(lat, 0.5), 2), "p99_ms": round(_pct(lat, 0.99), 2),
           "per_grid": per_grid_lat,
           "batched_solves_poisson": st_b["cohorts"], "largest_batch_poisson": st_b["largest_cohort"],
           "saturated": {"outstanding": outstanding, "solves_per_s": round(n_req / span_c, 4),
                         "vs_isolated": round(n_req / span_c / cap, 3),
                         "batched_solves": st_c["cohorts"],
                         "largest_batch": st_c["largest_cohort"],
                         "mean_batch": round(n_req / max(st_c["cohorts"], 1), 2)},
           "failed": st_b["failed"] + st_c["failed"], "peak_bytes": max(st_b["peak_bytes"],
                                                                        st_c["peak_bytes"]),
           "results_equal_alone": bool(same),
           "worst_last_change": max(errs),
           "worst_rel_res_true": max(info.rel_res_true for _, _, info in res_b + res_c)}
    log(f"[serve] {res}")
    return res


def batch_run(nrhs, tol, precond="prior"):
    """Multi-RHS batch: nrhs lognormal-Poisson catalogues of 1e6 galaxies on a
    shared 256^3 / 500 Mpc grid, mask and BBKS prior, CIC 2x supersampled,
    solved in one mixed-precision batch (every pass one launch for all RHS),
    with the catalogues already in HBM; per-iteration time and algorithmic
    bytes of the batched launches from the live profiler; compared with the
    same catalogues solved one at a time, and the PCIe-inclusive time from
    host catalogues."""
    import synth
    import torch
    import paper_0906_3978_amd as wf
    wl = synth.workload("bbks256")
    ptab = wl.ptab()
    w = wl.mask()
    cats = []
    t = time.perf_counter()
    for j in range(nrhs):
        wl.seed = 4000 + 3 * j
        cats.append(wl.catalogue(ptab, w).xyz)
    log(f"[batch] generated {nrhs} catalogues ({time.perf_counter() - t:.1f} s)")
    dev = torch.device("cuda:0")
    dcats = [torch.from_numpy(c).to(dev) for c in cats]
    outs = [torch.empty((wl.n,) * 3, dtype=torch.float64, device=dev) for _ in range(nrhs)]
    ctx = wf.Context(0)
    ctx.set_grid(wl.n, wl.box)
    ctx.set_mask(w)
    ctx.set_power(ptab)
    kw = dict(precision="mixed", tol=tol, max_iter=100000, precond=precond)
    ctx.solve_batch(dcats[:2], "cic", 2, outs=outs[:2], **kw)  # warm-up
    torch.cuda.synchronize()
    ctx.profile_enable(True)
    t = time.perf_counter()
    _, infos = ctx.solve_batch(dcats, "cic", 2, outs=outs, **kw)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    keys = SPLIT_F32 if precond == "prior" else PLAIN_F32
    it = _iteration_roofline(prof, keys, wl.n)
    if it:
        it["bytes_per_cell_per_rhs"] = round(it["bytes"] / (nrhs * wl.n ** 3), 2)
        it["model_ms_survey"] = round(76.25 * nrhs * wl.n ** 3 / (HBM_PEAK_GBS * 1e9) * 1e3, 3)
        it["model_ms_fold"] = round(68.0 * nrhs * wl.n ** 3 / (HBM_PEAK_GBS * 1e9) * 1e3, 3)
    t = time.perf_counter()
    singles = []
    one = torch.empty((wl.n,) * 3, dtype=torch.float64, device=dev)
    for xyz in dcats:
        ctx.set_galaxies(xyz)
        ctx.deposit("cic", 2)
        ctx.solve(out=one, **kw)
        singles.append(hashlib.sha256(one.cpu().numpy().tobytes()).hexdigest())
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t
    same = all(hashlib.sha256(o.cpu().numpy().tobytes()).hexdigest() == h
               for o, h in zip(outs, singles))
    t = time.perf_counter()
    ctx.solve_batch(cats, "cic", 2, **kw)
    t_host = time.perf_counter() - t
    iters = [i.iters_total for i in infos]
    res = {"nrhs": nrhs, "n": wl.n, "batch_s": round(t_batch, 3),
           "solves_per_s": round(nrhs / t_batch, 3), "sequential_s": round(t_single, 3),
           "speedup_batch_over_sequential": round(t_single / t_batch, 3),
           "iters_min_max": [min(iters), max(iters)],
           "iteration": it,
           "worst_last_change": max(i.last_change for i in infos),
           "worst_rel_res_true": max(i.rel_res_true for i in infos),
           "results_equal_single": bool(same),
           "host_catalogues_s": round(t_host, 3),
           "note": "batch_s and sequential_s with the catalogues in HBM; host_catalogues_s "
                   "includes the PCIe copies"}
    log(f"[batch] {res}")
    ctx.close()
    return res


def post_run(ctx, wl, field, reps=3):
    """The post-solve functions on the 512^3 solution already in HBM: RSD
    deconvolution (beta = 0.42, sigma = 500 km/s / H0, b = 1), Gaussian
    smoothing at r_S = 5 Mpc, masked moments, the inverse-weighting field of
    the same catalogue and the Sec. 4.1 measures between the two smoothed
    fields.  Each is timed on its own (device pointers, synchronised)."""
    import torch
    n = wl.n
    dec = torch.empty_like(field)
    sm = torch.empty_like(field)
    iw = torch.empty_like(field)
    iws = torch.empty_like(field)
    m = n ** 3

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            r = fn()
        torch.cuda.synchronize()
        return r, (time.perf_counter() - t) / reps

    beta, sigma = 0.42, 500.0 / 73.0
    _, t_rsd = timed(lambda: ctx.rsd_factor(beta, sigma))
    _, t_dec = timed(lambda: ctx.fourier_filter(field, "rsd_deconv", a=beta, b=sigma, c=1.0,
                                                out=dec))
    _, t_sm = timed(lambda: ctx.fourier_filter(dec, "gauss", a=5.0, out=sm))
    mom, t_mom = timed(lambda: ctx.field_moments(sm, masked=True))
    _, t_iw = timed(lambda: ctx.inverse_weighting(wl.scheme, wl.supersample, out=iw))
    ctx.fourier_filter(iw, "gauss", a=5.0, out=iws)
    cmp_, t_cmp = timed(lambda: ctx.compare_fields(sm, iws, masked=True))
    # FP64 bytes per cell of the five filter passes: the half spectrum is 8 B
    # per cell, so z R2C 8 + 8, y 8 + 8, x 8 + 8, y 8 + 8, z C2R 8 + 8; moments
    # read v and w, compare reads rec, truth and w
    filt_b, mom_b, cmp_b = 80 * m, 16 * m, 24 * m

    def gbs(b, t):
        return round(b / t / 1e9, 1)
    res = {"n": n, "reps": reps,
           "rsd_factor_ms": round(1e3 * t_rsd, 3),
           "rsd_deconv_ms": round(1e3 * t_dec, 3), "rsd_deconv_gbs": gbs(filt_b, t_dec),
           "gauss_ms": round(1e3 * t_sm, 3), "gauss_gbs": gbs(filt_b, t_sm),
           "moments_ms": round(1e3 * t_mom, 3), "moments_gbs": gbs(mom_b, t_mom),
           "inverse_weighting_ms": round(1e3 * t_iw, 3),
           "compare_ms": round(1e3 * t_cmp, 3), "compare_gbs": gbs(cmp_b, t_cmp),
           "filter_bytes_per_cell": 80,
           "moments_smoothed_masked": [round(x, 6) for x in mom],
           # D_KL is undefined (NaN) where 1 + delta <= 0: null in the JSON line
           "measures_wf_vs_iw_rs5": [round(x, 6) if math.isfinite(x) else None for x in cmp_]}
    log(f"[post] {res}")
    return res


def sd_run(nsamples, precond="prior", tol=1e-6):
    """Signal-dependent noise jackknife (Sec. 3.4): nsamples SD Wiener solves
    of one catalogue at the paper's mock-test size (128^3 / 500 Mpc, 2x
    supersampled CIC, BBKS prior, 60 deg cap), each with its own thinned
    noise estimate (alpha = 0.9 min w), mixed precision, solved 16 to a batch;
    the mean of the solutions is the estimate.  Also the flat-prior mean
    estimator (one solve) and the LSQ solve of the same data for reference."""
    import synth
    import torch
    import paper_0906_3978_amd as wf
    wl = synth.Workload("sd128", 128, 500.0, "cic", 2, 400_000, 7001, "bbks")
    ptab = wl.ptab()
    w = wl.mask()
    cat = wl.catalogue(ptab, w)
    dev = torch.device("cuda:0")
    ctx = wf.Context(0)
    ctx.set_grid(wl.n, wl.box)
    ctx.set_mask(torch.from_numpy(w).to(dev))
    ctx.set_power(torch.from_numpy(ptab).to(dev))
    ctx.set_galaxies(torch.from_numpy(cat.xyz).to(dev))
    ctx.deposit(wl.scheme, wl.supersample)
    mean = torch.empty((wl.n,) * 3, dtype=torch.float64, device=dev)
    alpha = 0.9 * float(w[w > 0].min())
    kw = dict(precision="mixed", precond=precond, tol=tol, max_iter=100000)
    ctx.solve_sd("jackknife", alpha=alpha, seed=11, nsamples=16, mean_out=mean, **kw)  # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, _, infos = ctx.solve_sd("jackknife", alpha=alpha, seed=11, nsamples=nsamples,
                               mean_out=mean, **kw)
    torch.cuda.synchronize()
    t_jk = time.perf_counter() - t
    t = time.perf_counter()
    _, _, minf = ctx.solve_sd("mean", mean_out=mean, **kw)
    torch.cuda.synchronize()
    t_mean = time.perf_counter() - t
    t = time.perf_counter()
    _, linf = ctx.solve(out=mean, **kw)
    torch.cuda.synchronize()
    t_lsq = time.perf_counter() - t
    iters = [i.iters_total for i in infos]
    res = {"n": wl.n, "n_gal": int(len(cat.xyz)), "nsamples": nsamples, "alpha": round(alpha, 4),
           "precond": precond, "tol": tol, "jackknife_s": round(t_jk, 3),
           "sd_solves_per_s": round(nsamples / t_jk, 2),
           "iters_min_max": [min(iters), max(iters)],
           "worst_rel_res_true": max(i.rel_res_true for i in infos),
           "sd_mean_estimator_s": round(t_mean, 4), "sd_mean_iters": minf[0].iters_total,
           "lsq_s": round(t_lsq, 4), "lsq_iters": linf.iters_total}
    log(f"[sd] {res}")
    ctx.close()
    return res


def deposit_run(n_gal, reps=5, seed=9100):
    """Deposit under contention (Sec. 3.1.2 mass assignment, int64 atomics):
    n_gal galaxies spread in four ways, from none to all on one point, on the
    serving mix's 128^3 grid (CIC, 2x supersampled: 256^3 fine nodes) and the
    headline 512^3 grid (TSC, 2x: 1024^3).  The time is the deposit class of
    the profiler (zero-fill of the fine grid + the atomic deposit); the empty
    catalogue gives the fill alone, so the difference is what the atomics
    cost.  Spreads: `uniform` in the box; `lognormal`, the BBKS lognormal-
    Poisson field of the grid (full sky); `blob`, a Gaussian of one fine cell's
    width around the box centre; `point`, every galaxy at one position (each
    of its 8 or 27 fine nodes takes n_gal atomic adds)."""
    import synth
    import torch
    import paper_0906_3978_amd as wf
    dev = torch.device("cuda:0")
    out = {}
    for n, scheme, box in ((128, "cic", 500.0), (512, "tsc", 500.0)):
        nf = 2 * n
        ptab = synth.p_by_m2(lambda k: synth.bbks_power(k), n, box)
        w = np.ones((n, n, n))
        rng = np.random.Generator(np.random.PCG64(seed + n))
        centre = 0.5 * box + 0.3 * box / nf
        blob = np.mod(centre + rng.normal(0.0, box / nf, size=(n_gal, 3)), box)
        blob[blob >= box] = 0.0
        cats = {"empty": np.zeros((0, 3)),
                "uniform": synth.uniform_catalogue(n_gal, box, seed + 1),
                "lognormal": synth.lognormal_catalogue(ptab, w, box, n_gal, seed + 2).xyz,
                "blob": np.ascontiguousarray(blob),
                "point": np.full((n_gal, 3), centre)}
        ctx = wf.Context(0)
        ctx.set_grid(n, box)
        ctx.set_mask(torch.from_numpy(w).to(dev))
        ctx.set_power(torch.from_numpy(ptab).to(dev))
        row = {}
        for name, xyz in cats.items():
            ctx.set_galaxies(torch.from_numpy(xyz).to(dev) if len(xyz) else xyz)
            ctx.deposit(scheme, 2)
            ctx.profile_enable(True)
            for _ in range(reps):
                ctx.deposit(scheme, 2)
            prof = ctx.profile_read()["deposit"]
            ctx.profile_enable(False)
            row[name] = {"n_gal": int(len(xyz)), "ms": round(prof["ms"] / prof["launches"], 4)}
        fill = row["empty"]["ms"]
        for name, r in row.items():
            if r["n_gal"]:
                r["atomics_ms"] = round(r["ms"] - fill, 4)
                r["ns_per_galaxy"] = round(1e6 * (r["ms"] - fill) / r["n_gal"], 3)
        out[f"{n}^3 {scheme} 2x"] = row
        log(f"[deposit] {n}^3 {scheme}: " + ", ".join(f"{k} {v['ms']:.3f} ms" for k, v in row.items()))
        ctx.close()
    return out


def traffic_for(kernel, launch_bytes):
    """HBM bytes per launch from committed rocprofv3 PMC counters, if they were
    taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    ent = t.get(kernel)
    if not ent or ent.get("kernel_hash") != kernel_hash():
        return None
    return ent.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="bbks512")
    ap.add_argument("--n", type=int, default=None, help="override the grid size (testing)")
    ap.add_argument("--tol", type=float, default=None,
                    help="outer residual tolerance (default: per --precond)")
    ap.add_argument("--inner-tol", type=float, default=0.0)
    ap.add_argument("--precond", choices=["none", "prior"], default="prior",
                    help="CG preconditioning: prior (the prior-split system C A C) or none "
                         "(plain CG on A)")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the comparison solve with plain (unpreconditioned) CG")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--profile-every", type=int, default=8,
                    help="live kernel timing over the timed steps: bracket one launch in this "
                         "many of each kernel class with events (1: every launch)")
    ap.add_argument("--profile-iters", type=int, default=0,
                    help="profiling run: one deposit, this many mixed iterations (of --precond) "
                         "and a 1 GiB device copy (the reference for scaling HBM counters), "
                         "then exit")
    ap.add_argument("--no-post", action="store_true",
                    help="skip timing the post-solve functions (filters, moments, IW)")
    ap.add_argument("--sd", type=int, default=200,
                    help="also run this many signal-dependent-noise jackknife solves at 128^3 "
                         "(0: skip)")
    ap.add_argument("--serve", type=int, default=60,
                    help="also run a serving stream of this many requests after 20 warm-up "
                         "requests, Poisson and saturated (0: skip)")
    ap.add_argument("--configs", type=int, default=1,
                    help="also run the plain FP64 configurations (32^3 power law, 256^3 BBKS) "
                         "with the oracle beside them (0: skip)")
    ap.add_argument("--deposit-stress", type=int, default=2_000_000,
                    help="also time the deposit of this many galaxies spread uniformly, "
                         "clustered and piled on one point, at 128^3 and 512^3 (0: skip)")
    ap.add_argument("--batch", type=int, default=16,
                    help="also run the multi-RHS batch: this many 256^3 catalogues in one solve "
                         "(0: skip)")
    args = ap.parse_args()
    if args.tol is None:
        args.tol = TOLERANCES[args.precond]

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(json.dumps({"error": "bench.py measures one GPU: the Wiener solve of one grid "
                          "runs on a single MI355X; run with --gpus 1"}))
        sys.exit(2)

    import torch
    import paper_0906_3978_amd as wf

    wl, ptab, w, cat = make_inputs(args.workload, args.n)
    n = wl.n
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ctx = wf.Context(0)
    xyz_d = torch.from_numpy(cat.xyz).to(dev)
    w_d = torch.from_numpy(w).to(dev)
    p_d = torch.from_numpy(ptab).to(dev)
    out = torch.empty((n, n, n), dtype=torch.float64, device=dev)
    ctx.set_grid(n, wl.box)
    ctx.set_mask(w_d)
    ctx.set_power(p_d)
    torch.cuda.synchronize()

    solve_kw = dict(precision="mixed", tol=args.tol, max_iter=100000, inner_tol=args.inner_tol,
                    precond=args.precond)

    if args.profile_iters:
        ctx.set_galaxies(xyz_d)
        ctx.deposit(wl.scheme, wl.supersample)
        _, info = ctx.solve(out=out, precision="mixed", tol=0.0, max_iter=args.profile_iters,
                            allow=(0, 5), precond=args.precond)
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile_iters": info.iters_total, "copy_bytes_each_way": 1 << 30}))
        return

    def step():
        ctx.set_galaxies(xyz_d)
        ctx.deposit(wl.scheme, wl.supersample)
        _, info = ctx.solve(out=out, **solve_kw)
        return info

    for i in range(args.warmup):
        t = time.perf_counter()
        info = step()
        log(f"[bench] warmup {i}: {time.perf_counter() - t:.3f} s, iters={info.iters_total} "
            f"outer={info.outer_steps} rel_res_true={info.rel_res_true:.2e}")

    if not args.no_profile:
        ctx.profile_enable(True, every=args.profile_every)
    torch.cuda.synchronize()
    lat = []
    infos = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        infos.append(step())
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = ctx.profile_read() if not args.no_profile else {}
    ctx.profile_enable(False)
    value = args.steps / elapsed
    info = infos[-1]
    log(f"[bench] timed {args.steps} steps in {elapsed:.3f} s: {value:.4f} solves/s; "
        f"iters={info.iters_total} outer={info.outer_steps} rel_res_true={info.rel_res_true:.2e}")

    # error of the last step's solution against the oracle's reference solution
    # of this workload (FP64 CG to 1e-12), stored as every 16th cell per axis
    err_ref = None
    ref_path = os.path.join(ROOT, "tests", "golden", f"{wl.name}_n{n}_x_s16.npy")
    if os.path.exists(ref_path):
        ref = np.load(ref_path).astype(np.float64)
        got = out[::16, ::16, ::16].cpu().numpy()
        err_ref = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        log(f"[bench] sampled rel. L2 error against the oracle reference: {err_ref:.3e}")

    roofline = None
    per_kernel = {}
    if prof:
        for k, v in prof.items():
            per_kernel[k] = dict(launches=v["launches"], skipped=v["skipped"],
                                 avg_us=round(1e3 * v["ms"] / v["launches"], 2),
                                 gbs=round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1) if v["ms"] > 0 else None)
        solve_kernels = {k: v for k, v in prof.items() if k not in ("deposit", "supersample")}
        dom = max(solve_kernels, key=lambda k: solve_kernels[k]["ms"])
        d = prof[dom]
        bpl = d["bytes"] / d["launches"]
        avg_s = d["ms"] * 1e-3 / d["launches"]
        ach = bpl / avg_s / 1e9
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                    "traffic": traffic_for(dom, bpl), "algorithmic_bytes_per_launch": bpl,
                    "avg_launch_us": round(avg_s * 1e6, 2)}
        # whole-iteration figure: the sweeps (+ update) of the FP32 inner CG
        it_keys = SPLIT_F32 if args.precond == "prior" else PLAIN_F32
        if all(k in prof for k in it_keys):
            it_ms = sum(prof[k]["ms"] / prof[k]["launches"] for k in it_keys)
            it_b = sum(prof[k]["bytes"] / prof[k]["launches"] for k in it_keys)
            roofline["iteration"] = {"ms": round(it_ms, 4), "bytes": it_b,
                                     "achieved": round(it_b / (it_ms * 1e-3) / 1e9, 1),
                                     "frac": round(it_b / (it_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                     "bytes_per_cell": round(it_b / n ** 3, 2)}

    fp64 = None
    if not args.no_fp64:
        ctx.set_galaxies(xyz_d)
        ctx.deposit(wl.scheme, wl.supersample)
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, inf64 = ctx.solve(out=out, precision="fp64", tol=args.tol, max_iter=100000,
                             precond=args.precond)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t
        fp64 = {"solve_s": round(t64, 4), "solves_per_s_solve_only": round(1.0 / t64, 4),
                "iters": inf64.iters_total, "rel_res_true": inf64.rel_res_true,
                "mixed_solve_s": round(info.time_ms * 1e-3, 4),
                "speedup_mixed_over_fp64_solve": round(t64 / (info.time_ms * 1e-3), 3)}
        log(f"[bench] fp64 solve {t64:.3f} s iters={inf64.iters_total}")

    plain = None
    if not args.no_plain and args.precond != "none":
        ctx.set_galaxies(xyz_d)
        ctx.deposit(wl.scheme, wl.supersample)
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, infp = ctx.solve(out=out, precision="mixed", tol=TOLERANCES["none"], max_iter=100000,
                            precond="none")
        torch.cuda.synchronize()
        tp = time.perf_counter() - t
        plain = {"precond": "none", "tol_outer": TOLERANCES["none"], "solve_s": round(tp, 4),
                 "iters": infp.iters_total, "outer_steps": infp.outer_steps,
                 "rel_res_true": infp.rel_res_true,
                 "speedup_of_prior_split": round(tp / (info.time_ms * 1e-3), 3)}
        log(f"[bench] plain mixed solve {tp:.3f} s iters={infp.iters_total}")
        # plain FP64 GPU CG (no preconditioning) to the same error target
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, inf64p = ctx.solve(out=out, precision="fp64", tol=TOLERANCES["none"], max_iter=100000,
                              precond="none")
        torch.cuda.synchronize()
        t64p = time.perf_counter() - t
        plain.update({"fp64_solve_s": round(t64p, 4), "fp64_iters": inf64p.iters_total,
                      "fp64_rel_res_true": inf64p.rel_res_true,
                      "speedup_mixed_prior_split_over_plain_fp64":
                          round(t64p / (info.time_ms * 1e-3), 3)})
        log(f"[bench] plain fp64 solve {t64p:.3f} s iters={inf64p.iters_total}")

    post = None
    if not args.no_post:
        ctx.set_galaxies(xyz_d)
        ctx.deposit(wl.scheme, wl.supersample)
        ctx.solve(out=out, **solve_kw)
        post = post_run(ctx, wl, out)

    cpu = None
    if not args.no_cpu_baseline:
        iters_ref = fp64["iters"] if fp64 else info.iters_total
        t = time.perf_counter()
        cpu = cpu_baseline(wl, ptab, w, cat.xyz, iters_ref, args.precond)
        log(f"[bench] cpu baseline {cpu['value']:.3e} solves/s on {cpu['cores']} threads "
            f"({time.perf_counter() - t:.1f} s): {cpu['sample']}")

    c1 = fp64_config_run("pl32", reps=5, cpu_full=True) if args.configs else None
    c2 = fp64_config_run("bbks256", reps=3) if args.configs else None

    serving = serve(args.serve, args.tol, args.precond) if args.serve else None
    batch = batch_run(args.batch, args.tol, args.precond) if args.batch else None
    sdres = sd_run(args.sd, args.precond) if args.sd else None
    dep = deposit_run(args.deposit_stress) if args.deposit_stress else None

    lat_ms = sorted(1e3 * x for x in lat)
    res = {
        "metric": "Wiener-CG solves/s at 512^3 to 1e-6 rel. L2 (mixed vs FP64); p50/p99 latency",
        "value": round(value, 5),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: {n}^3 grid, {wl.box:.0f} Mpc box, BBKS prior, "
                               f"60 deg cap x exp(-r/150 Mpc), {len(cat.xyz)} lognormal-Poisson "
                               f"galaxies, {wl.scheme.upper()} deposit 2x supersampled, "
                               f"mixed-precision "
                               f"{'prior-split ' if args.precond == 'prior' else ''}CG to "
                               f"FP64 residual {args.tol:g}",
                   "n": n, "box_mpc": wl.box, "n_gal": int(len(cat.xyz)),
                   "scheme": wl.scheme, "supersample": wl.supersample,
                   "precond": args.precond, "tol_outer": args.tol, "iters": info.iters_total,
                   "outer_steps": info.outer_steps, "rel_res_true": info.rel_res_true,
                   "rel_l2_error_vs_oracle_reference": err_ref,
                   "error_reference": "oracle FP64 CG to 1e-12, every 16th cell per axis "
                                      "(tests/golden)" if err_ref is not None else None},
        "latency_ms": {"p50": round(lat_ms[len(lat_ms) // 2], 3),
                       "p99": round(lat_ms[min(len(lat_ms) - 1, math.ceil(0.99 * len(lat_ms)) - 1)], 3)},
        "roofline": roofline,
        "kernels": per_kernel,
        "fp64": fp64,
        "plain_cg": plain,
        "post": post,
        "cpu_baseline": cpu,
        "c1_fp64_32": c1,
        "c2_fp64_256": c2,
        "serving": serving,
        "batch": batch,
        "signal_dependent": sdres,
        "deposit_contention": dep,
    }
    print(json.dumps(res))


if __name__ == "__main__":
    main()
