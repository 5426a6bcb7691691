"""The serving loop: requests of several grid sizes, masks and spectra
admitted by device-memory footprint; each result is bitwise the same alone
and in the mix, and matches the oracle."""
import numpy as np
import pytest

import synth
from oracle import wiener as ow

from gpu_util import rel_l2

pytestmark = pytest.mark.gpu

WF_OK, WF_EINVAL, WF_ENOMEM = 0, 1, 3


def _requests():
    reqs = []
    for i, n in enumerate([16, 32, 24, 48, 32, 16, 24]):
        wl = synth.serving_request(i, base_seed=900, box=300.0, grids=(n,))
        wl.n_target = min(wl.n_target, 40000)
        ptab = wl.ptab()
        w = wl.mask()
        cat = wl.catalogue(ptab, w)
        prec = "fp64" if i == 4 else "mixed"
        reqs.append(dict(n=n, box=wl.box, w=w, p=ptab, xyz=cat.xyz, prec=prec, wl=wl))
    return reqs


@pytest.fixture(scope="module")
def reqs():
    return _requests()


def _submit(srv, r):
    return srv.submit(r["n"], r["box"], r["w"], r["p"], r["xyz"], "cic", 2,
                      precision=r["prec"], tol=1e-10, max_iter=20000)


def test_mix_equals_alone_and_oracle(reqs):
    import paper_0906_3978_amd as wf
    alone = []
    with wf.Server(0, hbm_budget=2 << 30, max_active=1) as srv:
        for r in reqs:
            x, info = srv.wait(_submit(srv, r), r["n"])
            assert info.status == WF_OK, info
            alone.append(x)
    with wf.Server(0, hbm_budget=2 << 30, max_active=8) as srv:
        tickets = [_submit(srv, r) for r in reqs]
        mixed = [srv.wait(t, r["n"]) for t, r in zip(tickets, reqs)]
        st = srv.stats()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert 0 < st["p50_ms"] <= st["p99_ms"]
    assert st["peak_bytes"] > 0
    for a, (b, info) in zip(alone, mixed):
        assert info.status == WF_OK
        assert np.array_equal(a, b)
    # oracle check of two requests (one mixed, one FP64)
    for k in (0, 4):
        r = reqs[k]
        wl = r["wl"]
        res = ow.reconstruct(r["xyz"], wl.n, wl.box, r["w"], r["p"], "cic", 2, 1e-12, 20000)
        assert rel_l2(mixed[k][0], res["x"]) < 1e-6


def test_admission_by_footprint(reqs):
    import paper_0906_3978_amd as wf
    r = reqs[3]  # 48^3
    with wf.Server(0, hbm_budget=4 << 20, max_active=2) as srv:
        with pytest.raises(wf.WienerError) as e:
            _submit(srv, r)
        assert e.value.code == WF_ENOMEM
    # a budget that fits one 32^3 request at a time still serves a queue of them
    need = wf.footprint_bytes(32, 2, "mixed", 1)
    with wf.Server(0, hbm_budget=int(need * 1.6), max_active=4) as srv:
        ts = [_submit(srv, reqs[1]), _submit(srv, reqs[4]), _submit(srv, reqs[1])]
        outs = [srv.wait(t, 32) for t in ts]
    assert np.array_equal(outs[0][0], outs[2][0])


def test_invalid_and_cancel(reqs):
    import paper_0906_3978_amd as wf
    r = reqs[0]
    with wf.Server(0, hbm_budget=1 << 30, max_active=2) as srv:
        bad = r["w"].copy()
        bad[0, 0, 0] = 2.0
        with pytest.raises(wf.WienerError) as e:
            srv.submit(r["n"], r["box"], bad, r["p"], r["xyz"])
        assert e.value.code == WF_EINVAL
        t = _submit(srv, reqs[3])
        srv.cancel(t)
        done = False
        for _ in range(20000):
            done, info = srv.poll(t)
            if done:
                break
            import time
            time.sleep(0.001)
        assert done
        assert info.status in (WF_OK, 2)  # finished before the cancel, or cancelled
        srv.fetch(t, reqs[3]["n"], allow=(WF_OK, 2))


def test_served_requests_against_oracle():
    """Requests of the serving recipe at 64^3 and 128^3 (random cap, radial
    scale and prior amplitude; mixed prior-split CG to the split residual
    3e-7), served together: each result within 1e-6 relative L2 of the
    oracle's A^-1 b (its split CG to 1e-12)."""
    import paper_0906_3978_amd as wf
    reqs = []
    for i, n in enumerate([64, 128, 64]):
        wl = synth.serving_request(i, base_seed=7100, grids=(n,))
        wl.n_target = min(wl.n_target, 300_000)
        ptab = wl.ptab()
        w = wl.mask()
        reqs.append((wl, ptab, w, wl.catalogue(ptab, w).xyz))
    kw = dict(precision="mixed", precond="prior", tol=3e-7, max_iter=100000)
    with wf.Server(0, hbm_budget=4 << 30, max_active=4) as srv:
        tickets = [srv.submit(wl.n, wl.box, w, p, xyz, "cic", 2, **kw) for wl, p, w, xyz in reqs]
        got = [srv.wait(t, wl.n) for t, (wl, _, _, _) in zip(tickets, reqs)]
    for (wl, p, w, xyz), (x, info) in zip(reqs, got):
        assert info.status == WF_OK
        res = ow.reconstruct(xyz, wl.n, wl.box, w, p, "cic", 2, 0.0, 0, workers=16)
        ref = ow.split_cg(res["system"], res["b"], 1e-12, 100000)
        err = rel_l2(x, ref["x"])
        print(f"served {wl.n}^3: {len(xyz)} galaxies, {info.iters_total} iterations, "
              f"error {err:.3e}")
        assert err < 1e-6


def test_queued_requests_of_equal_kind_share_one_batched_solve():
    """With one batched solve in flight (max_active = 1), requests queued
    behind a long one are admitted together when it finishes: four 24^3
    requests with different masks, priors and catalogues form one cohort, and
    each result equals the same request served alone, bit for bit."""
    import paper_0906_3978_amd as wf
    big = synth.serving_request(0, base_seed=9100, box=300.0, grids=(64,))
    big.n_target = 300_000
    bp, bw = big.ptab(), big.mask()
    bxyz = big.catalogue(bp, bw).xyz
    small = []
    for i in range(4):
        wl = synth.serving_request(i + 1, base_seed=9100, box=300.0, grids=(24,))
        wl.n_target = min(wl.n_target, 30000)
        p, w = wl.ptab(), wl.mask()
        small.append((wl, p, w, wl.catalogue(p, w).xyz))
    kw = dict(precision="mixed", precond="prior", tol=1e-9, max_iter=100000)
    alone = []
    with wf.Server(0, hbm_budget=2 << 30, max_active=1) as srv:
        for wl, p, w, xyz in small:
            alone.append(srv.wait(srv.submit(wl.n, wl.box, w, p, xyz, "cic", 2, **kw), wl.n))
        assert srv.stats()["largest_cohort"] == 1
    with wf.Server(0, hbm_budget=2 << 30, max_active=1) as srv:
        tb = srv.submit(big.n, big.box, bw, bp, bxyz, "cic", 2, precision="fp64", tol=1e-12,
                        max_iter=100000)
        ts = [srv.submit(wl.n, wl.box, w, p, xyz, "cic", 2, **kw) for wl, p, w, xyz in small]
        xb, ib = srv.wait(tb, big.n)
        got = [srv.wait(t, wl.n) for t, (wl, _, _, _) in zip(ts, small)]
        st = srv.stats()
    print(f"cohorts {st['cohorts']}, largest {st['largest_cohort']}, big solve "
          f"{ib.iters_total} iterations")
    assert ib.status == WF_OK
    assert st["cohorts"] == 2 and st["largest_cohort"] == 4
    for (xa, ia), (xg, ig) in zip(alone, got):
        assert ig.status == WF_OK
        assert ig.iters_total == ia.iters_total
        assert np.array_equal(xa, xg)


def test_small_requests_do_not_wait_behind_large_ones():
    """With two streams, one running a 192^3 solve, the last free stream is
    kept for small grids: a 32^3 request submitted after a second 192^3 one
    is served at once, while the second large request waits for the first."""
    import paper_0906_3978_amd as wf
    reqs = []
    for i, n in enumerate([192, 192, 32]):
        wl = synth.serving_request(i, base_seed=9300, box=400.0, grids=(n,))
        wl.n_target = min(wl.n_target, 200_000)
        p, w = wl.ptab(), wl.mask()
        reqs.append((wl, p, w, wl.catalogue(p, w).xyz))
    kw = dict(precision="mixed", precond="prior", tol=1e-6, max_iter=100000)
    with wf.Server(0, hbm_budget=16 << 30, max_active=2) as srv:
        ts = [srv.submit(wl.n, wl.box, w, p, xyz, "cic", 2, **kw) for wl, p, w, xyz in reqs]
        got = [srv.wait(t, wl.n) for t, (wl, _, _, _) in zip(ts, reqs)]
        st = srv.stats()
    (_, l1), (_, l2), (_, s) = got
    print(f"latency ms: large {l1.latency_ms:.1f}, {l2.latency_ms:.1f}; small {s.latency_ms:.1f}")
    assert all(i.status == WF_OK for _, i in got)
    assert st["cohorts"] == 3 and st["failed"] == 0
    assert s.latency_ms < l1.latency_ms < l2.latency_ms
