"""CPU oracle for the C-AMS pressure solve — TEST INFRASTRUCTURE ONLY.

Thin ctypes wrapper around `cams_oracle.c` (plain FP64 C).  Only the tests,
the smoke check and the CPU-baseline leg of the benchmark may import this
package; the GPU library never does, and this package never imports the GPU
library.  See `cams_oracle.c` for the equations each function follows.

Parity status: every function here is pinned by `-m "not gpu"` tests
(closed forms, invariants, SciPy/NumPy direct solves); none is "unpinned".
"""

from __future__ import annotations

import contextlib
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


_TIMING_LIB = os.path.join(_HERE, "libcams_oracle_omp.so")


def build_timing() -> str:
    """The CPU-baseline timing build of the same source: -O3 -march=native
    -fopenmp (the loops marked "omp parallel" run on all host cores; see the
    header of cams_oracle.c).  Built on the machine that runs it, since
    -march=native targets that machine's CPU."""
    tmp = _TIMING_LIB + ".tmp"
    subprocess.check_call(["gcc", "-O3", "-march=native", "-fopenmp", "-std=c99", "-fPIC", "-shared",
                           "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, _TIMING_LIB)
    return _TIMING_LIB


@contextlib.contextmanager
def timing_build(threads: int):
    """Run the oracle functions of this module on the timing build with
    `threads` OpenMP threads (build it first with build_timing())."""
    global _lib
    saved = _lib
    L = _configure(ctypes.CDLL(_TIMING_LIB))
    L.omp_set_num_threads(int(threads))
    _lib = L
    try:
        yield L
    finally:
        _lib = saved


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = _configure(ctypes.CDLL(_LIB))
    return _lib


def _configure(L):
    """Result and argument types of the oracle entry points."""
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
    return L


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


def face_bc_arrays(pb):
    """(bt, bp) of the Dirichlet boundary faces of pb.face_bc ({"W": p, "E": p}
    for the west face x = 0 / east face x = nx - 1), or (None, None):
    bt = half-cell transmissibility 2 (k / mu) dy dz / dx of a cell whose
    face lies on such a boundary, bp = the face pressure."""
    bc = getattr(pb, "face_bc", None)
    if not bc:
        return None, None
    bt = np.zeros(pb.n)
    bp = np.zeros(pb.n)
    i = np.arange(pb.n) % pb.nx
    for side, col in (("W", 0), ("E", pb.nx - 1)):
        if side in bc:
            m = i == col
            bt[m] = 2.0 * np.asarray(pb.perm)[m] / pb.mu * pb.dy * pb.dz / pb.dx
            bp[m] = float(bc[side])
    return bt, bp


def _bc_ptrs(pb):
    bt, bp = face_bc_arrays(pb)
    if bt is None:
        return None, None, ()
    return _ptr(bt), _ptr(bp), (bt, bp)


def nonlinear_residual(pb, T, p, pn):
    """(F, ||eps||_2): mass-form residual of Eq. (2) and the error norm."""
    g, f = grid_of(pb), fluid_of(pb)
    F = np.zeros(pb.n)
    q = None if pb.q is None else _f64(pb.q)
    dm = pb.dirichlet_mask()
    T = _f64(T)
    btp, bpp, keep = _bc_ptrs(pb)
    e = lib().or_nonlinear_residual(ctypes.byref(g), ctypes.byref(f), _ptr(T[0]), _ptr(T[1]),
                                    _ptr(T[2]), _ptr(_f64(pb.phi)),
                                    None if q is None else _ptr(q), _ptr(dm), btp, bpp,
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
    btp, bpp, keep = _bc_ptrs(pb)
    e = lib().or_linear_system(ctypes.byref(g), ctypes.byref(f), _ptr(T[0]), _ptr(T[1]), _ptr(T[2]),
                               _ptr(_f64(pb.phi)), None if q is None else _ptr(q), _ptr(dm), btp, bpp,
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


def basis_general(pb, C, adiag=None) -> np.ndarray:
    """Slot-major basis (8, N) of the local operator with face couplings C
    (3, N) and extra diagonal adiag (N,) or None (Eqs. (8)-(11))."""
    g = grid_of(pb)
    C = _f64(C)
    P = np.zeros((8, pb.n))
    rc = lib().or_basis_general(ctypes.byref(g), _ptr(C[0]), _ptr(C[1]), _ptr(C[2]),
                                None if adiag is None else _ptr(_f64(adiag)), _ptr(P))
    if rc != 0:
        raise RuntimeError("oracle basis construction failed")
    return P


B4, B3, B2, B1 = 0, 3, 2, 1


def basis_operator(pb, T, kind, p=None, pn=None):
    """(couplings (3, N), extra diagonal or None) of the local problems of
    basis type `kind` (Sec. 3), in the mass form of the Newton system:
      B4  -div(lambda grad Phi) = 0:           couplings T;
      B3  c^n Phi - div(lambda grad Phi) = 0:  couplings T, diagonal phi c dV / dt
          (c^n at the old time: phi/dt d(ln rho)/dp = phi c / dt);
      B2  -(1/rho) div(rho lambda grad Phi) = 0, times rho dV: couplings
          W = T (rho_i + rho_j)/2 at the iterate p (no Dirichlet masking);
      B1  c Phi - (1/rho) div(rho lambda grad Phi) = 0, times rho dV:
          couplings W and the accumulation diagonal of the Newton matrix,
          phi c rho(pn) dV / dt."""
    T = np.asarray(T, dtype=np.float64)
    dV = pb.dx * pb.dy * pb.dz
    if kind == B4:
        return T, None
    if kind == B3:
        return T, pb.phi * pb.c * dV / pb.dt * np.ones(pb.n)
    rho = (pb.rho0 * np.exp(pb.c * (np.asarray(p) - pb.p0))).reshape(pb.nz, pb.ny, pb.nx)
    W = np.zeros_like(T)
    for a, axis in ((0, 2), (1, 1), (2, 0)):
        hi = [slice(None)] * 3
        hi[axis] = slice(1, None)
        nb = np.zeros_like(rho)
        lo = [slice(None)] * 3
        lo[axis] = slice(0, -1)
        nb[tuple(lo)] = rho[tuple(hi)]
        W[a] = (T[a].reshape(rho.shape) * 0.5 * (rho + nb)).reshape(-1)
    if kind == B2:
        return W, None
    rhon = pb.rho0 * np.exp(pb.c * (np.asarray(pn) - pb.p0))
    return W, pb.phi * pb.c * rhon * dV / pb.dt


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
SMOOTH_NATURAL = 3     # ILU(0) of the whole matrix in natural (lexicographic) order


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
               rtol=None, maxit=None, atol=None):
    """(d, iterations, history): C-AMS iteration on A d = r0.  `ilu` is one
    smoother, or a pair whose members the Richardson steps of each smoothing
    stage take in turn (first, second, first, ...)."""
    g = grid_of(pb)
    W = _f64(W)
    n_pre = pb.n_pre if n_pre is None else n_pre
    n_post = pb.n_post if n_post is None else n_post
    rtol = pb.lin_rtol if rtol is None else rtol
    maxit = pb.lin_maxit if maxit is None else maxit
    atol = getattr(pb, "lin_atol", 0.0) if atol is None else atol
    first, alt = (ilu[0], ilu[1]) if isinstance(ilu, (tuple, list)) else (ilu, None)
    d = np.zeros(pb.n)
    hist = np.zeros(maxit + 1)
    its = lib().or_cams_solve(ctypes.byref(g), _ptr(W[0]), _ptr(W[1]), _ptr(W[2]), _ptr(_f64(diag)),
                              _ptr(pb.dirichlet_mask()), _ptr(_f64(P)), int(restriction),
                              _ptr(LU), _ptr(piv), ctypes.c_void_p(first.h),
                              ctypes.c_void_p(alt.h if alt is not None else None), int(n_pre), int(n_post),
                              ctypes.c_double(rtol), ctypes.c_double(atol), int(maxit), _ptr(_f64(r0)), _ptr(d),
                              _ptr(hist))
    n_hist = (its + 1) if its >= 0 else (maxit + 1)
    return d, its, hist[:n_hist]


def smoother_for(pb, W, diag, smoother=None):
    """The ILU(0) smoother the problem asks for (default: block-Jacobi): one
    ILU0, or for SMOOTH_BLOCK_ALT the pair (blocks at the origin, shifted
    blocks); for SMOOTH_NATURAL the global ILU(0) in cell order; otherwise
    the red-black order."""
    kind = getattr(pb, "smoother", SMOOTH_BLOCK) if smoother is None else smoother
    if kind == SMOOTH_BLOCK:
        return ILU0(pb, W, diag, block=smoother_block(pb))
    if kind == SMOOTH_BLOCK_ALT:
        return (ILU0(pb, W, diag, block=smoother_block(pb)),
                ILU0(pb, W, diag, block=smoother_block(pb), shift=smoother_shift(pb)))
    if kind == SMOOTH_NATURAL:
        return ILU0(pb, W, diag, order=np.arange(pb.n, dtype=np.int64))
    return ILU0(pb, W, diag)


def newton_step(pb, T, P, pn, p, restriction=None, n_pre=None, n_post=None, lin_rtol=None,
                lin_maxit=None, newton_tol=None, newton_maxit=None, smoother=None, lin_atol=None):
    """One time step.  Returns (p_new, status, stats dict)."""
    g, f = grid_of(pb), fluid_of(pb)
    T = _f64(T)
    p = np.array(p, dtype=np.float64, copy=True)
    q = None if pb.q is None else _f64(pb.q)
    st = np.zeros(3)
    kind = getattr(pb, "smoother", SMOOTH_BLOCK) if smoother is None else smoother
    btp, bpp, keep = _bc_ptrs(pb)
    rc = lib().or_newton_step(
        ctypes.byref(g), ctypes.byref(f), _ptr(T[0]), _ptr(T[1]), _ptr(T[2]), _ptr(_f64(pb.phi)),
        None if q is None else _ptr(q), _ptr(pb.dirichlet_mask()), btp, bpp, _ptr(_f64(P)),
        int(pb.restriction if restriction is None else restriction),
        int(pb.n_pre if n_pre is None else n_pre), int(pb.n_post if n_post is None else n_post),
        ctypes.c_double(pb.lin_rtol if lin_rtol is None else lin_rtol),
        ctypes.c_double(getattr(pb, "lin_atol", 0.0) if lin_atol is None else lin_atol),
        int(pb.lin_maxit if lin_maxit is None else lin_maxit),
        ctypes.c_double(pb.newton_tol if newton_tol is None else newton_tol),
        int(pb.newton_maxit if newton_maxit is None else newton_maxit),
        int({SMOOTH_BLOCK: 1, SMOOTH_BLOCK_ALT: 2, SMOOTH_NATURAL: 3}.get(kind, 0)), *smoother_block(pb),
        _ptr(_f64(pn)), _ptr(p), _ptr(st))
    return p, rc, {"newton_iters": int(st[0]), "lin_iters": int(st[1]), "eps_norm": float(st[2])}


def full_dual_blocks(pb) -> np.ndarray:
    """(B, 3) first interior cell (x, y, z) of every full dual block: the
    7x7x7 cells strictly between two vertex planes 8 cells apart on every
    axis (Sec. 3 dual grid; vertices from `vertex_coords`).  Order: x
    fastest, then y, then z."""
    starts = []
    for n, r in ((pb.nx, pb.rx), (pb.ny, pb.ry), (pb.nz, pb.rz)):
        v = vertex_coords(n, r)
        starts.append([int(v[a]) + 1 for a in range(len(v) - 1) if v[a + 1] - v[a] == 8])
    out = [(x, y, z) for z in starts[2] for y in starts[1] for x in starts[0]]
    return np.array(out, dtype=np.int64).reshape(-1, 3)


def basis_block_ratios(pb, T, P, starts) -> np.ndarray:
    """Local-equation check of the basis on full dual blocks: for each block,
    sqrt(sum_s sum_{i in I} ((T Phi_s)_i)^2 / sum_s sum_{i in I} (T_IF Phi_s)_i^2),
    with I the 7^3 interior cells, T the incompressible two-point operator
    of Eq. (11) (type B4: zero row sums), Phi_s the basis function of the
    block's corner node s (s = bx + 2 by + 4 bz) and T_IF the couplings of an
    interior cell to the block's boundary cells (its bounding vertex planes).
    Zero for the exact local solve; one when the interior values are zero.

    P is slot-major: P[s][n] belongs to the node s relative to cell n's lower
    bracketing vertex (the largest vertex coordinate <= the cell's, per
    axis).  Interior cells and the lower vertex planes share the block's
    lower vertex; on an upper vertex plane the lower vertex is the block's
    upper one, so node s of the block is slot s - bit there when s has that
    axis' bit, and otherwise a node whose function vanishes on that plane."""
    T = np.asarray(T, dtype=np.float64)
    nx, ny, nz = pb.nx, pb.ny, pb.nz
    Tx, Ty, Tz = (T[a].reshape(nz, ny, nx) for a in range(3))
    Pg = np.asarray(P, dtype=np.float64).reshape(8, nz, ny, nx)
    out = np.zeros(len(starts))
    for b, (x0, y0, z0) in enumerate(starts):
        # the 9x9x9 patch: interior at patch positions 1..7, vertex planes at 0 and 8
        zs, ys, xs = slice(z0 - 1, z0 + 8), slice(y0 - 1, y0 + 8), slice(x0 - 1, x0 + 8)
        ext = np.zeros((8, 9, 9, 9))
        for s in range(8):
            ext[s] = Pg[s, zs, ys, xs]
        for s in range(8):
            # upper vertex planes: node s of the block is stored under slot s - bit
            for axis, bit in ((2, 1), (1, 2), (0, 4)):    # patch axes (z, y, x) and slot bits
                sl = [slice(None)] * 3
                sl[axis] = 8
                sl = tuple(sl)
                ext[s][sl] = Pg[s - bit, zs, ys, xs][sl] if s & bit else 0.0
        tx = Tx[z0 - 1:z0 + 8, y0 - 1:y0 + 8, x0 - 1:x0 + 8]
        ty = Ty[z0 - 1:z0 + 8, y0 - 1:y0 + 8, x0 - 1:x0 + 8]
        tz = Tz[z0 - 1:z0 + 8, y0 - 1:y0 + 8, x0 - 1:x0 + 8]
        I = slice(1, 8)
        num = den = 0.0
        for s in range(8):
            e = ext[s]
            c = e[I, I, I]
            # (neighbour values, face transmissibility, interior cells whose neighbour is a boundary cell)
            faces = ((e[I, I, 0:7], tx[I, I, 0:7], (slice(None), slice(None), 0)),
                     (e[I, I, 2:9], tx[I, I, 1:8], (slice(None), slice(None), 6)),
                     (e[I, 0:7, I], ty[I, 0:7, I], (slice(None), 0, slice(None))),
                     (e[I, 2:9, I], ty[I, 1:8, I], (slice(None), 6, slice(None))),
                     (e[0:7, I, I], tz[0:7, I, I], (0, slice(None), slice(None))),
                     (e[2:9, I, I], tz[1:8, I, I], (6, slice(None), slice(None))))
            res = np.zeros((7, 7, 7))
            bnd = np.zeros((7, 7, 7))
            for nb, tf, edge in faces:
                res += tf * (c - nb)
                bnd[edge] += (tf * nb)[edge]
            num += float((res ** 2).sum())
            den += float((bnd ** 2).sum())
        out[b] = np.sqrt(num / den) if den > 0 else 0.0
    return out


def newton_history(pb, T, P, pn, p, lin_rtol, newton_tol, lin_atol=0.0, newton_maxit=30, lin_maxit=2000):
    """Error and residual norm histories of one time step (Sec. 4.1.1, Table
    "conv" and its adaptive variant): Newton iterations of the paper's
    linearisation, each solved by C-AMS to ||r|| <= max(lin_rtol ||r0||,
    lin_atol); after every C-AMS iteration i of Newton iteration nu the
    entry (nu, ||r_i||_2, ||eps(p^nu + d_i)||_2) is recorded, i = 0 being the
    start of the solve.  d_i is obtained by running the C-AMS solve from
    zero for exactly i iterations (the iteration is deterministic), so the
    cost is quadratic in the iteration count: small grids only.
    Returns (p, nu (n,), res (n,), err (n,))."""
    p = np.array(p, dtype=np.float64, copy=True)
    nus, res, err = [], [], []
    for nu in range(newton_maxit + 1):
        W, diag, r0, e = linear_system(pb, T, p, pn)
        if e <= newton_tol:
            return p, np.array(nus), np.array(res), np.array(err)
        LU, piv = lu_factor(coarse_operator(pb, W, diag, P, pb.restriction))
        ilu = smoother_for(pb, W, diag)
        d_full, its, _ = cams_solve(pb, W, diag, P, pb.restriction, LU, piv, ilu, r0, rtol=lin_rtol,
                                    atol=lin_atol, maxit=lin_maxit)
        if its < 0:
            raise RuntimeError("oracle linear solve did not converge")
        for i in range(its + 1):
            if i == its:
                d = d_full
            else:
                d, _, _ = cams_solve(pb, W, diag, P, pb.restriction, LU, piv, ilu, r0, rtol=0.0, atol=0.0,
                                     maxit=i)
            nus.append(nu)
            res.append(float(np.linalg.norm(r0 - matvec(pb, W, diag, d))))
            err.append(nonlinear_residual(pb, T, p + d, pn)[1])
        p = p + d_full
    raise RuntimeError("oracle Newton did not converge")


def face_flux(pb, T, p, p_rho=None):
    """(3, N) two-point mass fluxes on the +x/+y/+z face of every cell:
    T (rho_n + rho_m)/2 (p_n - p_m), positive out of the cell, 0 on the domain
    boundary; densities at p_rho (default p: the fluxes of F(p); the
    assembled iterate: the fluxes of that Newton linear system)."""
    g, f = grid_of(pb), fluid_of(pb)
    T = _f64(T)
    F = np.zeros((3, pb.n))
    q = _f64(p if p_rho is None else p_rho)
    lib().or_face_flux(ctypes.byref(g), ctypes.byref(f), _ptr(T[0]), _ptr(T[1]), _ptr(T[2]), _ptr(q),
                       _ptr(_f64(p)), _ptr(F[0]), _ptr(F[1]), _ptr(F[2]))
    return F


def conservative_sweep(pb, T, P, p, pn):
    """One MSFV multiscale stage after a converged MSFE solve (Sec. 4.2: use
    MSFE to converge, then a single MSFV sweep for mass conservation; MSFV
    gives locally conservative fluxes after its multiscale stage, Sec. 4):
    assemble the Newton system at p, form R^FV A P_hat (Eq. (13) with the
    restriction of Eq. (7)), solve the coarse system for R^FV r (LU with
    partial pivoting), prolong (Eq. (12)) and update; the fluxes are those
    of the assembled linear system at the updated pressure (face densities
    at p), which balance the linearised accumulation on every coarse block.
    Returns (p_new, d, fluxes (3, N))."""
    W, diag, r0, _ = linear_system(pb, T, p, pn)
    LU, piv = lu_factor(coarse_operator(pb, W, diag, P, FV))
    xc = lu_solve(LU, piv, restrict(pb, P, FV, r0))
    d = prolong(pb, P, xc)
    p_new = np.asarray(p, dtype=np.float64) + d
    return p_new, d, face_flux(pb, T, p_new, p_rho=p)


def cell_outflow(pb, F):
    """Net outflow of every cell from the (3, N) face fluxes: its own +x/+y/+z
    fluxes minus those of its -x/-y/-z neighbours."""
    nx, ny, nz = pb.nx, pb.ny, pb.nz
    out = np.zeros((nz, ny, nx))
    for a, axis in ((0, 2), (1, 1), (2, 0)):
        Fa = np.asarray(F[a]).reshape(nz, ny, nx)
        out += Fa
        sl_hi = [slice(None)] * 3
        sl_lo = [slice(None)] * 3
        sl_hi[axis] = slice(1, None)
        sl_lo[axis] = slice(0, -1)
        out[tuple(sl_hi)] -= Fa[tuple(sl_lo)]
    return out.reshape(-1)


def block_balance(pb, T, p, pn):
    """Per primal coarse block, the sum of the mass-form residual F over its
    cells: accumulation + net outflow through the block's boundary - sources
    (Eq. (2) integrated over the block; interior faces cancel)."""
    F, _ = nonlinear_residual(pb, T, p, pn)
    return np.bincount(primal_block(pb), weights=F, minlength=num_coarse(pb))


def newton_step_basis(pb, T, pn, p, kind, lin_rtol, newton_tol, newton_maxit=30, lin_maxit=2000):
    """One time step with basis type `kind` (Sec. 3): B3/B4 built once at
    the start, B1/B2 rebuilt from the current iterate at every Newton
    iteration (Table "cams" step 3; every region, i.e. a zero update
    threshold).  Returns (p, Newton iterations, C-AMS iterations)."""
    p = np.array(p, dtype=np.float64, copy=True)
    P = None
    lits = 0
    for nu in range(newton_maxit + 1):
        W, diag, r0, e = linear_system(pb, T, p, pn)
        if e <= newton_tol:
            return p, nu, lits
        if P is None or kind in (B1, B2):
            P = basis_general(pb, *basis_operator(pb, T, kind, p=p, pn=pn))
        LU, piv = lu_factor(coarse_operator(pb, W, diag, P, pb.restriction))
        d, its, _ = cams_solve(pb, W, diag, P, pb.restriction, LU, piv, smoother_for(pb, W, diag), r0,
                               rtol=lin_rtol, maxit=lin_maxit)
        if its < 0:
            raise RuntimeError("oracle linear solve did not converge")
        lits += its
        p = p + d
    raise RuntimeError("oracle Newton did not converge")
