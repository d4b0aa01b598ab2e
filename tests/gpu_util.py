"""Helpers of the GPU parity tests (the HIP path through the C ABI)."""

from __future__ import annotations

import numpy as np
import pytest


def require_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no ROCm GPU visible")
    from paper_1705_05783_amd import _cams
    _cams.load()   # raises if the HIP library is missing: no fallback
    return torch


def to_np(t):
    return t.detach().cpu().numpy()


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    scale = max(np.max(np.abs(b)), 1e-300)
    return float(np.max(np.abs(a - b)) / scale)


def solver_for(pb, **kw):
    from paper_1705_05783_amd.solver import Solver
    return Solver(pb, **kw)


def log(*args):
    print(*args, flush=True)
