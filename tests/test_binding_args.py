"""The Python binding refuses arrays whose dtype, size or device differ from
what the C ABI will read or write, before any call into the library (CPU; the
library is replaced by a recorder, so nothing reaches a GPU)."""
import numpy as np
import pytest
import torch

import paper_0906_3978_amd as wf
from paper_0906_3978_amd import _lib


class Recorder:
    """Stands in for the loaded library: every entry point records its call."""

    def __init__(self):
        self.calls = []

    def __getattr__(self, name):
        def f(*args):
            self.calls.append(name)
            return 0
        return f


def _ctx(n=8):
    c = wf.Context.__new__(wf.Context)
    c._L = Recorder()
    c._h = None
    c.device = 0
    c.n, c.box = n, 100.0
    return c


def test_arg_accepts_matching_arrays():
    a = np.zeros(12)
    assert _lib._arg(a, "f64", 12, "a")[1] == _lib.WF_HOST
    t = torch.zeros(4, 3, dtype=torch.float64)
    assert _lib._arg(t, "f64", 12, "t")[0] == t.data_ptr()
    assert _lib._arg(np.zeros(5, dtype=np.int32), "i32", 5, "c")[1] == _lib.WF_HOST
    assert _lib._arg(None, "f64", 3, "none") == (None, _lib.WF_HOST)


@pytest.mark.parametrize("bad,err", [
    (np.zeros(12, dtype=np.float32), TypeError),
    (np.zeros(11), ValueError),
    (torch.zeros(12, dtype=torch.float32), TypeError),
    (torch.zeros(13, dtype=torch.float64), ValueError),
    ([0.0] * 12, TypeError),
])
def test_arg_refuses_mismatches(bad, err):
    with pytest.raises(err):
        _lib._arg(bad, "f64", 12, "x")


def test_solve_refuses_a_wrong_output():
    c = _ctx()
    with pytest.raises(TypeError):
        c.solve(out=np.empty((8, 8, 8), dtype=np.float32))
    with pytest.raises(ValueError):
        c.solve(out=np.empty((8, 8, 7)))
    with pytest.raises(TypeError):
        c.solve(out=torch.empty((8, 8, 8), dtype=torch.float32))
    assert c._L.calls == []


def test_inputs_of_the_wrong_size_are_refused():
    c = _ctx()
    with pytest.raises(ValueError):
        c.set_mask(np.ones((8, 8, 9)))
    with pytest.raises(TypeError):
        c.set_power(torch.ones(49, dtype=torch.float32))
    with pytest.raises(ValueError):
        c.set_galaxies(np.zeros(7))
    with pytest.raises(ValueError):
        c.set_rhs(np.zeros(100), 1.0)
    with pytest.raises(ValueError):
        c.inverse_weighting(out=np.empty(10))
    with pytest.raises(TypeError):
        c.jackknife_counts(0.5, 1, count=2, out=np.empty((2, 8, 8, 8), dtype=np.int64))
    with pytest.raises(ValueError):
        c.solve_sd(mean_out=np.empty((8, 8, 8)), samples_out=np.empty((1, 8, 8, 8)),
                   nsamples=2, kind="jackknife")
    with pytest.raises(ValueError):
        c.fourier_filter(np.zeros((8, 8, 8)), "gauss", out=np.empty((4, 4, 4)))
    with pytest.raises(ValueError):
        c.compare_fields(np.zeros((8, 8, 8)), np.zeros((4, 4, 4)))
    with pytest.raises(ValueError):
        c.solve_batch([np.zeros((3, 3))], outs=[np.empty((4, 4, 4))])
    assert c._L.calls == []


def test_matching_inputs_reach_the_library():
    c = _ctx()
    c.set_mask(np.ones((8, 8, 8)))
    c.set_rhs(np.zeros((8, 8, 8)), 1.0)
    c.solve(out=np.empty((8, 8, 8)))
    assert c._L.calls == ["wf_set_mask", "wf_set_rhs", "wf_solve"]


def test_server_fetch_uses_the_request_grid():
    s = wf.Server.__new__(wf.Server)
    s._L = Recorder()
    s._h = None
    s._grid = {7: 16}
    with pytest.raises(ValueError):
        s.fetch(7, 8)
    with pytest.raises(ValueError):
        s.fetch(9)
    with pytest.raises(ValueError):
        s.submit(16, 100.0, np.ones((8, 8, 8)), np.ones(193), np.zeros((0, 3)))
    assert s._L.calls == []
