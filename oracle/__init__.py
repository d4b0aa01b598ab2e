"""CPU oracle for the C-AMS pressure solve — TEST INFRASTRUCTURE ONLY.

Thin ctypes wrapper around `cams_oracle.c` (plain FP64 C).  Only the tests,
the smoke check and the CPU-baseline leg of the benchmark may import this
package; the GPU library never does, and this package never imports the GPU
library.  See `cams_oracle.c` for the equations each function follows.

Parity status: every function here is pinned by `-m "not gpu"` tests
(closed forms, invariants, SciPy/NumPy direct solves); none is "unpinned".
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cams_oracle.c")
_LIB = os.path.join(_HERE, "libcams_oracle.so")

FV = 0
FE = 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, FP64, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fno-fast-math",
                               "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("rx", ctypes.c_int32), ("ry", ctypes.c_int32), ("rz", ctypes.c_int32)]


class _Fluid(ctypes.Structure):
    _fields_ = [("rho0", ctypes.c_double), ("c", ctypes.c_double), ("p0", ctypes.c_double),
                ("mu", ctypes.c_double), ("dt", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L.or_nonlinear_residual.restype = ctypes.c_double
        L.or_linear_system.restype = ctypes.c_double
        L.or_basis_b4.restype = ctypes.c_int
        L.or_num_coarse.restype = ctypes.c_int
        L.or_num_blocks.restype = ctypes.c_int
        L.or_lu_factor.restype = ctypes.c_int
        L.or_ilu0_create.restype = P
        L.or_ilu0_create.argtypes = [P, P, P, P, P, P]
        L.or_ilu0_block_create.restype = P
        L.or_ilu0_block_create.argtypes = [P, P, P, P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.or_ilu0_block_create_shifted.restype = P
        L.or_ilu0_block_create_shifted.argtypes = [P, P, P, P, P] + [ctypes.c_int] * 6
        L.or_ilu0_free.argtypes = [P]
        L.or_ilu0_nnz.restype = ctypes.c_long
        L.or_ilu0_nnz.argtypes = [P]
        L.or_ilu0_export.argtypes = [P, P, P, P]
        L.or_ilu0_apply.argtypes = [P, P, P]
        L.or_cams_solve.restype = ctypes.c_int
        L.or_newton_step.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def grid_of(pb) -> _Grid:
    return _Grid(pb.nx, pb.ny, pb.nz, pb.dx, pb.dy, pb.dz, pb.rx, pb.ry, pb.rz)


def fluid_of(pb) -> _Fluid:
    return _Fluid(pb.rho0, pb.c, pb.p0, pb.mu, pb.dt)


def num_coarse(pb) -> int:
    g = grid_of(pb)
    return lib().or_num_coarse(ctypes.byref(g))


def vertex_coords(n: int, r: int) -> np.ndarray:
    nb = lib().or_num_blocks(n, r)
    v = np.zeros(nb, dtype=np.int32)
    lib().or_vertex_coords(n, r, _ptr(v))
    return v


def transmissibility(pb):
    """(Tx, Ty, Tz) two-point face transmissibilities, each (N,)."""
    g = grid_of(pb)
    N = pb.n
    T = np.zeros((3, N))
    lib().or_transmissibility(ctypes.byref(g), ctypes.c_double(pb.mu), _ptr(_f64(pb.perm)),
                              _ptr(T[0]), _ptr(T[1]), _ptr(T[2]))
    return T


def nonlinear_residual(pb, T, p, pn):
    """(F, ||eps||_2): mass-form residual of Eq. (2) and the error norm."""
    g, f = grid_of(pb), fluid_of(pb)
    F = np.zeros(pb.n)
    q = None if pb.q is None else _f64(pb.q)
    dm = pb.dirichlet_mask()
    T = _f64(T)
    e = lib().or_nonlinear_residual(ctypes.byref(g), ctypes.byref(f), _ptr(T[0]), _ptr(T[1]),
                                    _ptr(T[2]), _ptr(_f64(pb.phi)),
                                    None if q is None else _ptr(q), _ptr(dm),
                                    _ptr(_f64(p)), _ptr(_f64(pn)), _ptr(F))
    return F, e


def linear_system(pb, T, p, pn):
    """(W (3,N), diag (N,), r (N,), ||eps||_2) of one Newton iteration."""
    g, f = grid_of(pb), fluid_of(pb)
    N = pb.n
    W = np.zeros((3, N))
    diag = np.zeros(N)
    r = np.zeros(N)
    q = None if pb.q is None else _f64(pb.q)
    dm = pb.dirichlet_mask()
    T = _f64(T)
    e = lib().or_linear_system(ctypes.byref(g), ctypes.byref(f), _ptr(T[0]), _ptr(T[1]), _ptr(T[2]),
                               _ptr(_f64(pb.phi)), None if q is None else _ptr(q), _ptr(dm),
                               _ptr(_f64(p)), _ptr(_f64(pn)),
                               _ptr(W[0]), _ptr(W[1]), _ptr(W[2]), _ptr(diag), _ptr(r))
    return W, diag, r, e


def matvec(pb, W, diag, x):
    g = grid_of(pb)
    W = _f64(W)
    y = np.zeros(pb.n)
    lib().or_matvec(ctypes.byref(g), _ptr(W[0]), _ptr(W[1]), _ptr(W[2]), _ptr(_f64(diag)),
                    _ptr(_f64(x)), _ptr(y))
    return y


def cell_levels(pb) -> np.ndarray:
    g = grid_of(pb)
    lv = np.zeros(pb.n, dtype=np.int32)
    lib().or_cell_levels(ctypes.byref(g), _ptr(lv))
    return lv


def basis_b4(pb, T) -> np.ndarray:
    """Slot-major basis weights P (8, N) of type B4."""
    g = grid_of(pb)
    T = _f64(T)
    P = np.zeros((8, pb.n))
    rc = lib().or_basis_b4(ctypes.byref(g), _ptr(T[0]), _ptr(T[1]), _ptr(T[2]), _ptr(P))
    if rc != 0:
        raise RuntimeError("oracle basis construction failed")
    return P


def slot_nodes(pb) -> np.ndarray:
    """(8, N) coarse node index of each slot, -1 where absent."""
    g = grid_of(pb)
    nodes = np.zeros((8, pb.n), dtype=np.int32)
    lib().or_slot_nodes(ctypes.byref(g), _ptr(nodes))
    return nodes


def primal_block(pb) -> np.ndarray:
    g = grid_of(pb)
    b = np.zeros(pb.n, dtype=np.int32)
    lib().or_primal_block(ctypes.byref(g), _ptr(b))
    return b


def coarse_operator(pb, W, diag, P, restriction) -> np.ndarray:
    g = grid_of(pb)
    Nc = num_coarse(pb)
    Ac = np.zeros((Nc, Nc))
    W = _f64(W)
    lib().or_coarse_operator(ctypes.byref(g), _ptr(W[0]), _ptr(W[1]), _ptr(W[2]), _ptr(_f64(diag)),
                             _ptr(pb.dirichlet_mask()), _ptr(_f64(P)), int(restriction), _ptr(Ac))
    return Ac


def restrict(pb, P, restriction, x) -> np.ndarray:
    g = grid_of(pb)
    xc = np.zeros(num_coarse(pb))
    lib().or_restrict(ctypes.byref(g), _ptr(pb.dirichlet_mask()), _ptr(_f64(P)), int(restriction),
                      _ptr(_f64(x)), _ptr(xc))
    return xc


def prolong(pb, P, xc) -> np.ndarray:
    g = grid_of(pb)
    x = np.zeros(pb.n)
    lib().or_prolong(ctypes.byref(g), _ptr(pb.dirichlet_mask()), _ptr(_f64(P)), _ptr(_f64(xc)), _ptr(x))
    return x


def lu_factor(A):
    LU = np.array(A, dtype=np.float64, order="C", copy=True)
    n = LU.shape[0]
    piv = np.zeros(n, dtype=np.int32)
    if lib().or_lu_factor(n, _ptr(LU), _ptr(piv)) != 0:
        raise np.linalg.LinAlgError("singular coarse matrix")
    return LU, piv


def lu_solve(LU, piv, b):
    x = np.array(b, dtype=np.float64, copy=True)
    lib().or_lu_solve(LU.shape[0], _ptr(LU), _ptr(piv), _ptr(x))
    return x


def redblack_order(pb) -> np.ndarray:
    g = grid_of(pb)
    o = np.zeros(pb.n, dtype=np.int64)
    lib().or_redblack_order(ctypes.byref(g), _ptr(o))
    return o


SMOOTH_BLOCK = 0       # block-Jacobi ILU(0), natural order inside 8x8x8 blocks
SMOOTH_REDBLACK = 1    # ILU(0) in red-black order
SMOOTH_BLOCK_ALT = 2   # block ILU(0), every other step on the half-block-shifted block grid


def smoother_block(pb):
    """Smoother block extents: 8 cells per active axis."""
    return (8, 8, 8 if pb.nz > 1 else 1)


def smoother_shift(pb):
    """Offsets of the shifted block grid: half a block per active axis."""
    return tuple(b // 2 for b in smoother_block(pb))


class ILU0:
    """ILU(0) of the 7-point operator: in a given ordering (default
    red-black), or block-Jacobi ILU(0) when `block` = (bx, by, bz), on the
    block grid shifted cyclically by `shift` = (ox, oy, oz) cells."""

    def __init__(self, pb, W, diag, order=None, block=None, shift=(0, 0, 0)):
        self.pb = pb
        g = grid_of(pb)
        W = _f64(W)
        self._keep = (W, _f64(diag))
        if block is not None:
            self.order = np.arange(pb.n, dtype=np.int64)
            self.h = lib().or_ilu0_block_create_shifted(ctypes.byref(g), _ptr(W[0]), _ptr(W[1]), _ptr(W[2]),
                                                        _ptr(self._keep[1]), int(block[0]), int(block[1]),
                                                        int(block[2]), int(shift[0]), int(shift[1]),
                                                        int(shift[2]))
            return
        self.order = redblack_order(pb) if order is None else np.ascontiguousarray(order, dtype=np.int64)
        self.h = lib().or_ilu0_create(ctypes.byref(g), _ptr(W[0]), _ptr(W[1]), _ptr(W[2]),
                                      _ptr(self._keep[1]), _ptr(self.order))

    def apply(self, z):
        x = np.zeros(self.pb.n)
        lib().or_ilu0_apply(self.h, _ptr(_f64(z)), _ptr(x))
        return x

    def export(self):
        nnz = lib().or_ilu0_nnz(self.h)
        rp = np.zeros(self.pb.n + 1, dtype=np.int64)
        col = np.zeros(nnz, dtype=np.int64)
        val = np.zeros(nnz)
        lib().or_ilu0_export(self.h, _ptr(rp), _ptr(col), _ptr(val))
        return rp, col, val

    def __del__(self):
        try:
            lib().or_ilu0_free(self.h)
        except Exception:
            pass


def cams_solve(pb, W, diag, P, restriction, LU, piv, ilu, r0, n_pre=None, n_post=None,
               rtol=None, maxit=None):
    """(d, iterations, history): C-AMS iteration on A d = r0.  `ilu` is one
    smoother, or a pair whose members the Richardson steps of each smoothing
    stage take in turn (first, second, first, ...)."""
    g = grid_of(pb)
    W = _f64(W)
    n_pre = pb.n_pre if n_pre is None else n_pre
    n_post = pb.n_post if n_post is None else n_post
    rtol = pb.lin_rtol if rtol is None else rtol
    maxit = pb.lin_maxit if maxit is None else maxit
    first, alt = (ilu[0], ilu[1]) if isinstance(ilu, (tuple, list)) else (ilu, None)
    d = np.zeros(pb.n)
    hist = np.zeros(maxit + 1)
    its = lib().or_cams_solve(ctypes.byref(g), _ptr(W[0]), _ptr(W[1]), _ptr(W[2]), _ptr(_f64(diag)),
                              _ptr(pb.dirichlet_mask()), _ptr(_f64(P)), int(restriction),
                              _ptr(LU), _ptr(piv), ctypes.c_void_p(first.h),
                              ctypes.c_void_p(alt.h if alt is not None else None), int(n_pre), int(n_post),
                              ctypes.c_double(rtol), int(maxit), _ptr(_f64(r0)), _ptr(d), _ptr(hist))
    n_hist = (its + 1) if its >= 0 else (maxit + 1)
    return d, its, hist[:n_hist]


def smoother_for(pb, W, diag, smoother=None):
    """The ILU(0) smoother the problem asks for (default: block-Jacobi): one
    ILU0, or for SMOOTH_BLOCK_ALT the pair (blocks at the origin, shifted
    blocks)."""
    kind = getattr(pb, "smoother", SMOOTH_BLOCK) if smoother is None else smoother
    if kind == SMOOTH_BLOCK:
        return ILU0(pb, W, diag, block=smoother_block(pb))
    if kind == SMOOTH_BLOCK_ALT:
        return (ILU0(pb, W, diag, block=smoother_block(pb)),
                ILU0(pb, W, diag, block=smoother_block(pb), shift=smoother_shift(pb)))
    return ILU0(pb, W, diag)


def newton_step(pb, T, P, pn, p, restriction=None, n_pre=None, n_post=None, lin_rtol=None,
                lin_maxit=None, newton_tol=None, newton_maxit=None, smoother=None):
    """One time step.  Returns (p_new, status, stats dict)."""
    g, f = grid_of(pb), fluid_of(pb)
    T = _f64(T)
    p = np.array(p, dtype=np.float64, copy=True)
    q = None if pb.q is None else _f64(pb.q)
    st = np.zeros(3)
    kind = getattr(pb, "smoother", SMOOTH_BLOCK) if smoother is None else smoother
    rc = lib().or_newton_step(
        ctypes.byref(g), ctypes.byref(f), _ptr(T[0]), _ptr(T[1]), _ptr(T[2]), _ptr(_f64(pb.phi)),
        None if q is None else _ptr(q), _ptr(pb.dirichlet_mask()), _ptr(_f64(P)),
        int(pb.restriction if restriction is None else restriction),
        int(pb.n_pre if n_pre is None else n_pre), int(pb.n_post if n_post is None else n_post),
        ctypes.c_double(pb.lin_rtol if lin_rtol is None else lin_rtol),
        int(pb.lin_maxit if lin_maxit is None else lin_maxit),
        ctypes.c_double(pb.newton_tol if newton_tol is None else newton_tol),
        int(pb.newton_maxit if newton_maxit is None else newton_maxit),
        int({SMOOTH_BLOCK: 1, SMOOTH_BLOCK_ALT: 2}.get(kind, 0)), *smoother_block(pb),
        _ptr(_f64(pn)), _ptr(p), _ptr(st))
    return p, rc, {"newton_iters": int(st[0]), "lin_iters": int(st[1]), "eps_norm": float(st[2])}
