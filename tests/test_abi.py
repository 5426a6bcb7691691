"""Host-side checks of the C-ABI library: it loads, exports every entry point
include/wiener.h declares, and its host-only functions behave."""
import ctypes
import os
import re

import pytest

import paper_0906_3978_amd as wf

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "wiener.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wf_[a-z0-9_]+)\s*\(", text)) - {"wf_alloc_fn", "wf_free_fn"})


def test_every_declared_symbol_is_exported():
    L = ctypes.CDLL(wf.LIB_PATH)
    names = _declared()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_header():
    assert set(_declared()) == set(wf.SIGNATURES)


def test_version_and_status_strings():
    L = wf.lib()
    assert L.wf_abi_version() == 3
    for code in range(8):
        assert L.wf_status_str(code)
    assert b"unknown" in L.wf_status_str(99)


def test_footprint_model():
    f = wf.footprint_bytes
    assert f(64, 2, "mixed", 1) < f(128, 2, "mixed", 1) < f(256, 2, "mixed", 1)
    assert f(256, 2, "mixed", 16) > 10 * f(256, 1, "mixed", 1) / 2
    # 512^3 mixed with the 2x deposit stays far below one GPU's 288 GB
    assert 8e9 < f(512, 2, "mixed", 1) < 64e9
    assert f(0, 2, "mixed", 1) == 0
    assert f(64, 3, "mixed", 1) == 0


def test_null_context_is_rejected():
    L = wf.lib()
    assert L.wf_set_grid(None, 32, 100.0) == 1
    assert L.wf_ctx_destroy(None) == 1
    assert L.wf_last_error(None) == b"null context"
