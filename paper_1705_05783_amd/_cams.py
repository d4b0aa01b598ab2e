"""ctypes binding of libcams.so: the C ABI of include/cams.h, same names.

Argument marshalling only; every step of the solve runs in the HIP library.
Importing this module raises if the library has not been built.
"""

from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcams.so")

CAMS_OK = 0
CAMS_E_ARG = -1
CAMS_E_STATE = -2
CAMS_E_DEVICE = -3
CAMS_E_NOMEM = -4
CAMS_E_NOT_CONVERGED = -5
CAMS_E_BREAKDOWN = -6

CAMS_R_FV = 0
CAMS_R_FE = 1
CAMS_FP64 = 0
CAMS_MIXED_FP32 = 1
CAMS_MIXED_BF16 = 2
CAMS_SMOOTH_BLOCK_ILU0 = 0
CAMS_SMOOTH_RB_ILU0 = 1
CAMS_SMOOTH_BLOCK_ALT_ILU0 = 2
CAMS_SMOOTH_NAT_ILU0 = 3

CAMS_ARR_T = 0
CAMS_ARR_W = 1
CAMS_ARR_DIAG = 2
CAMS_ARR_R0 = 3
CAMS_ARR_P = 4
CAMS_ARR_AC = 5
CAMS_ARR_AC_INV = 6
CAMS_ARR_INVD = 7

CAMS_BASIS_B4 = 0
CAMS_BASIS_B1 = 1
CAMS_BASIS_B2 = 2
CAMS_BASIS_B3 = 3
CAMS_PROF_NONE = 0
CAMS_PROF_SMOOTH_STEP = 1


class cams_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("rx", ctypes.c_int32), ("ry", ctypes.c_int32), ("rz", ctypes.c_int32)]


class cams_fluid(ctypes.Structure):
    _fields_ = [("rho0", ctypes.c_double), ("c", ctypes.c_double), ("p0", ctypes.c_double),
                ("mu", ctypes.c_double), ("dt", ctypes.c_double)]


class cams_options(ctypes.Structure):
    _fields_ = [("restriction", ctypes.c_int32), ("n_pre", ctypes.c_int32), ("n_post", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("smoother", ctypes.c_int32),
                ("lin_rtol", ctypes.c_double), ("lin_maxit", ctypes.c_int32),
                ("newton_tol", ctypes.c_double), ("newton_maxit", ctypes.c_int32),
                ("lin_atol", ctypes.c_double), ("basis_type", ctypes.c_int32), ("basis_tol", ctypes.c_double),
                ("coarse_tol", ctypes.c_double)]


class cams_stats(ctypes.Structure):
    _fields_ = [("newton_iters", ctypes.c_int32), ("lin_iters_total", ctypes.c_int32),
                ("lin_iters_last", ctypes.c_int32), ("fallback_blocks", ctypes.c_int32),
                ("relres_last", ctypes.c_double), ("eps_norm_last", ctypes.c_double),
                ("t_assemble_ms", ctypes.c_double), ("t_basis_ms", ctypes.c_double),
                ("t_coarse_ms", ctypes.c_double), ("t_iterate_ms", ctypes.c_double),
                ("basis_updates", ctypes.c_int32), ("basis_regions_rebuilt", ctypes.c_int32),
                ("coarse_factorizations", ctypes.c_int32), ("basis_rebuilds", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


# (name, restype, argtypes) for every entry point declared in include/cams.h
_VP = ctypes.c_void_p
_I = ctypes.c_int
_SIGS = [
    ("cams_create", _I, [ctypes.POINTER(cams_grid), ctypes.POINTER(cams_fluid), ctypes.POINTER(cams_options),
                         _VP, ctypes.POINTER(_VP)]),
    ("cams_workspace_bytes", ctypes.c_size_t, [_VP]),
    ("cams_set_workspace", _I, [_VP, _VP, ctypes.c_size_t]),
    ("cams_set_rock", _I, [_VP, _VP, _VP, _VP]),
    ("cams_set_wells", _I, [_VP, _VP, _VP, ctypes.c_int32]),
    ("cams_assemble", _I, [_VP, _VP, _VP, ctypes.POINTER(ctypes.c_double)]),
    ("cams_build_basis", _I, [_VP]),
    ("cams_coarse_op", _I, [_VP]),
    ("cams_iterate", _I, [_VP, _VP, ctypes.POINTER(cams_stats)]),
    ("cams_newton_step", _I, [_VP, _VP, _VP, ctypes.POINTER(cams_stats)]),
    ("cams_conservative_sweep", _I, [_VP, _VP, _VP, _VP]),
    ("cams_set_face_dirichlet", _I, [_VP, ctypes.c_int32, ctypes.c_double]),
    ("cams_newton_history", _I, [_VP, _VP, _VP, _VP, _VP, _VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                 ctypes.POINTER(cams_stats)]),
    ("cams_smooth_apply", _I, [_VP, _VP, _VP]),
    ("cams_array_bytes", ctypes.c_size_t, [_VP, _I]),
    ("cams_export", _I, [_VP, _I, _VP, ctypes.c_size_t]),
    ("cams_import_basis", _I, [_VP, _VP, ctypes.c_size_t]),
    ("cams_num_coarse", ctypes.c_int64, [_VP]),
    ("cams_debug_gemm_sub", _I, [_VP, _VP, _VP, _VP, _I, _I, _I]),
    ("cams_cnn_num_params", ctypes.c_int64, []),
    ("cams_cnn_workspace_bytes", ctypes.c_size_t, [ctypes.c_int32]),
    ("cams_cnn_forward", _I, [_VP, _VP, _VP, ctypes.c_int32, _VP, _VP]),
    ("cams_cnn_bf16_workspace_bytes", ctypes.c_size_t, []),
    ("cams_cnn_forward_bf16", _I, [_VP, _VP, _VP, ctypes.c_int32, _VP, _VP]),
    ("cams_cnn_noalloc_scratch_bytes", ctypes.c_size_t, []),
    ("cams_cnn_forward_bf16_noalloc", _I, [_VP, _VP, _VP, ctypes.c_int32, _VP]),
    ("cams_cnn_loss_grad", _I, [_VP, _VP, _VP, _VP, ctypes.c_int32, _VP, _VP, _VP]),
    ("cams_cnn_adam", _I, [_VP, _VP, _VP, _VP, _VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                           ctypes.c_float, ctypes.c_float, ctypes.c_float]),
    ("cams_cnn_num_blocks", ctypes.c_int32, [_VP]),
    ("cams_cnn_patches", _I, [_VP, _VP, _VP]),
    ("cams_learned_scratch_bytes", ctypes.c_size_t, [_VP]),
    ("cams_set_learned", _I, [_VP, _VP, _VP, ctypes.c_size_t, ctypes.c_double]),
    ("cams_set_learned_guard", _I, [_VP, ctypes.c_int32]),
    ("cams_basis_stats", _I, [_VP, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    ("cams_basis_block_ratios", _I, [_VP, _VP, ctypes.c_int32]),
    ("cams_profile", _I, [_VP, _I]),
    ("cams_profile_read", _I, [_VP, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                               ctypes.POINTER(ctypes.c_double)]),
    ("cams_destroy", _I, [_VP]),
    ("cams_status_string", ctypes.c_char_p, [_I]),
    ("cams_last_error", ctypes.c_char_p, [_VP]),
    ("cams_invalidate_basis", _I, [_VP]),
    ("cams_coarse_planes", ctypes.c_int32, [_VP]),
    ("cams_debug_coarse_solve", _I, [_VP, _VP, _VP]),
    ("cams_batch_create", _I, [ctypes.POINTER(_VP), ctypes.c_int32, _VP, ctypes.POINTER(_VP)]),
    ("cams_batch_workspace_bytes", ctypes.c_size_t, [_VP]),
    ("cams_batch_set_workspace", _I, [_VP, _VP, ctypes.c_size_t]),
    ("cams_batch_newton_iteration", _I, [_VP, ctypes.POINTER(_VP), ctypes.POINTER(_VP),
                                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(cams_stats)]),
    ("cams_batch_tuning", _I, [_VP, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                               ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double),
                               ctypes.POINTER(ctypes.c_double), ctypes.c_int32]),
    ("cams_batch_set_smoother", _I, [_VP, ctypes.c_int32, ctypes.c_int32]),
    ("cams_batch_tuning_source", _I, [_VP, ctypes.POINTER(ctypes.c_int32)]),
    ("cams_batch_clear_tuning_cache", None, []),
    ("cams_batch_last_error", ctypes.c_char_p, [_VP]),
    ("cams_batch_destroy", None, [_VP]),
]

EXPORTED = [name for name, _, _ in _SIGS]

_lib = None


def load():
    """Load libcams.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                              "python paper_1705_05783_amd/build.py")
        lib = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class CamsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def check(status, ctx=None, what=""):
    if status != CAMS_OK:
        lib = load()
        detail = lib.cams_last_error(ctx).decode() if ctx else lib.cams_status_string(status).decode()
        raise CamsError(status, f"{what}: {detail}")
    return status


def _fwd(name):
    def f(*args):
        return getattr(load(), name)(*args)
    f.__name__ = name
    return f


# one forwarder per entry point of include/cams.h, e.g. cams_iterate(...)
for _name in EXPORTED:
    globals()[_name] = _fwd(_name)
del _name
