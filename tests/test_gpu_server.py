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
