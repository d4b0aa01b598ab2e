"""The allocation-free inference entry point against the workspace one.

cams_cnn_forward_bf16_noalloc runs the learned basis' matrix-core inference
with its weight workspace in a static device array; its output must equal
cams_cnn_forward_bf16's (same kernels, same arithmetic: bit for bit) on two
calls in a row, the second with a smaller batch, and on a third call with
different weights after those (the array keeps the last call's contents).
"""

import ctypes

import numpy as np
import pytest

from tests.gpu_util import log, require_gpu, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _noalloc_fn():
    from paper_1705_05783_amd import _cams as C
    return C.cams_cnn_forward_bf16_noalloc


def _with_workspace(torch, params, feat):
    from paper_1705_05783_amd import learned
    return learned.forward(params, feat, bf16=True)


def _noalloc(torch, fn, params, feat):
    phi = torch.empty((feat.shape[0], 8, 729), dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    rc = fn(ctypes.c_void_p(st), ctypes.c_void_p(params.data_ptr()), ctypes.c_void_p(feat.data_ptr()),
            int(feat.shape[0]), ctypes.c_void_p(phi.data_ptr()))
    assert rc == 0, rc
    torch.cuda.synchronize()
    return phi


def test_noalloc_inference_matches_workspace_entry_point(torch):
    from paper_1705_05783_amd import _cams as C
    from paper_1705_05783_amd import learned
    from paper_1705_05783_amd.train_basis import load_weights
    fn = _noalloc_fn()
    log("bf16 workspace bytes", C.cams_cnn_bf16_workspace_bytes(), "fixed array", C.cams_cnn_noalloc_scratch_bytes())
    assert C.cams_cnn_bf16_workspace_bytes() <= C.cams_cnn_noalloc_scratch_bytes()
    rng = np.random.default_rng(3)
    trained = load_weights()
    other = learned.init_params(5)
    cases = [(trained, 37), (trained, 5), (other, 11)]
    for params, batch in cases:
        feat = torch.tensor(rng.normal(size=(batch, 3, 729)), dtype=torch.float32, device="cuda")
        ref = to_np(_with_workspace(torch, params, feat))
        got = to_np(_noalloc(torch, fn, params, feat))
        log("batch", batch, "max |diff|", float(np.abs(got - ref).max()))
        assert got.shape == ref.shape and np.array_equal(got, ref)
    # a batch of 0 is rejected on the host, before any device work
    phi = torch.empty(8, dtype=torch.float32, device="cuda")
    rc = fn(ctypes.c_void_p(0), ctypes.c_void_p(trained.data_ptr()), ctypes.c_void_p(phi.data_ptr()), 0,
            ctypes.c_void_p(phi.data_ptr()))
    assert rc == C.CAMS_E_ARG
