"""Shared helpers of the GPU tests (contexts, workloads, comparisons)."""
import numpy as np
import pytest


def context():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("a GPU is required for tests marked gpu")
    import paper_0906_3978_amd as wf
    return wf.Context(0)


def rel_max(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def rel_l2(a, b):
    d = np.asarray(a, dtype=np.float64) - b
    return float(np.sqrt((d * d).sum() / (np.asarray(b) ** 2).sum()))
