"""Batched solve of many independent problems (libcams cams_batch_* calls).

All solvers of a batch share one stream; torch provides the batch's device
workspace.  One call advances every instance by one Newton iteration with
the C-AMS iterations of all instances fused into one launch per kernel.
"""

from __future__ import annotations

import ctypes

import torch

from . import _cams as C
from .solver import Solver


def _check(status, b, what):
    if status != C.CAMS_OK:
        detail = C.cams_batch_last_error(b).decode() if b else C.cams_status_string(status).decode()
        raise C.CamsError(status, f"{what}: {detail}")


class Batch:
    def __init__(self, solvers):
        self.solvers = list(solvers)
        if not self.solvers:
            raise ValueError("empty batch")
        self.device = self.solvers[0].device
        self.stream = self.solvers[0].stream
        arr = (ctypes.c_void_p * len(self.solvers))(*[s.ctx.value for s in self.solvers])
        h = ctypes.c_void_p()
        _check(C.cams_batch_create(arr, len(self.solvers), ctypes.c_void_p(self.stream.cuda_stream),
                                   ctypes.byref(h)), None, "cams_batch_create")
        self.handle = h
        nbytes = C.cams_batch_workspace_bytes(h)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        _check(C.cams_batch_set_workspace(h, ctypes.c_void_p(ptr), nbytes), h, "cams_batch_set_workspace")

    @classmethod
    def from_problems(cls, problems, device="cuda:0"):
        stream = torch.cuda.current_stream(torch.device(device))
        return cls([Solver(pb, device=device, stream=stream) for pb in problems])

    def newton_iteration(self, pn, p, check=True):
        """pn, p: lists of device FP64 pressure tensors (p updated in place).
        Returns (per-instance status list, per-instance stats dicts)."""
        n = len(self.solvers)
        if len(pn) != n or len(p) != n:
            raise ValueError("one pressure pair per instance")
        for t in list(pn) + list(p):
            if not (t.is_contiguous() and t.dtype == torch.float64 and t.device == self.device):
                raise ValueError("pressures must be contiguous float64 tensors on the batch device")
        pa = (ctypes.c_void_p * n)(*[t.data_ptr() for t in pn])
        pb = (ctypes.c_void_p * n)(*[t.data_ptr() for t in p])
        st = (ctypes.c_int32 * n)()
        stats = (C.cams_stats * n)()
        status = C.cams_batch_newton_iteration(self.handle, pa, pb, st, stats)
        if check and status != C.CAMS_OK and status not in (C.CAMS_E_NOT_CONVERGED, C.CAMS_E_BREAKDOWN):
            _check(status, self.handle, "cams_batch_newton_iteration")
        return list(st), [s.as_dict() for s in stats]

    def set_smoother(self, threads, blocks):
        """Fix the smoother form ((128|256|512, 1), or (512, 4) in mixed
        precision); (0, 0) returns to the tuner's choice."""
        _check(C.cams_batch_set_smoother(self.handle, int(threads), int(blocks)), self.handle,
               "cams_batch_set_smoother")

    def tuning(self):
        k, nt, nb = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        ms, sm = (ctypes.c_double * 4)(), (ctypes.c_double * 4)()
        _check(C.cams_batch_tuning(self.handle, ctypes.byref(k), ctypes.byref(nt), ctypes.byref(nb), ms, sm, 4),
               self.handle, "cams_batch_tuning")
        src = ctypes.c_int32()
        _check(C.cams_batch_tuning_source(self.handle, ctypes.byref(src)), self.handle, "cams_batch_tuning_source")
        return {"iters_per_graph": k.value, "smoother_threads": nt.value, "smoother_blocks": nb.value,
                "ms_per_iter": list(ms)[:3], "ms_per_smooth_step": list(sm), "from_cache": src.value}

    @staticmethod
    def clear_tuning_cache():
        """Forget the tuning outcomes stored by earlier batches of this process."""
        C.cams_batch_clear_tuning_cache()

    def close(self):
        if self.handle:
            C.cams_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
