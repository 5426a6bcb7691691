"""The allocation-free moments entry point against the allocating one, through
the C ABI: the same bits on two calls in a row, the second on a smaller grid,
masked and unmasked; a host pointer is refused before any kernel runs."""
import ctypes

import numpy as np
import pytest

import synth

from gpu_util import context

pytestmark = pytest.mark.gpu

WF_OK, WF_EINVAL, WF_DEVICE = 0, 1, 1


def _both(ctx, v, masked):
    import paper_0906_3978_amd as wf
    L = wf.lib()
    a = np.full(5, -1.0)
    b = np.full(5, -2.0)
    assert L.wf_field_moments(ctx._h, v.data_ptr(), int(masked), a.ctypes.data, WF_DEVICE) == WF_OK
    assert L.wf_field_moments_noalloc(ctx._h, v.data_ptr(), int(masked), b.ctypes.data) == WF_OK
    return a, b


def test_noalloc_moments_equal_the_allocating_entry_point():
    import torch
    ctx = context()
    try:
        for n, seed in ((48, 1), (24, 2)):
            box = 4.0 * n
            ctx.set_grid(n, box)
            ctx.set_mask(synth.cap_mask(n, box, 65.0, 0.5 * box))
            g = torch.Generator(device="cpu").manual_seed(seed)
            v = torch.randn((n, n, n), dtype=torch.float64, generator=g).exp().to("cuda:0")
            for masked in (False, True):
                a, b = _both(ctx, v, masked)
                print(f"{n}^3 masked={masked}: {a}")
                assert np.array_equal(a, b)
                assert a[0] > 0 and (masked or a[0] == n ** 3)
                ref = v.double().cpu().numpy().ravel()
                if not masked:
                    assert a[1] == pytest.approx(ref.mean(), rel=1e-12)
                    assert a[2] == pytest.approx(ref.var(), rel=1e-10)
    finally:
        ctx.close()


def test_noalloc_moments_refuse_host_memory():
    import paper_0906_3978_amd as wf
    ctx = context()
    try:
        n = 16
        ctx.set_grid(n, 100.0)
        host = np.ones((n, n, n))
        out = np.zeros(5)
        assert wf.lib().wf_field_moments_noalloc(ctx._h, host.ctypes.data, 0,
                                                 out.ctypes.data) == WF_EINVAL
        assert not out.any()
    finally:
        ctx.close()
