"""Convenience wrapper over the libcams C ABI for one problem on one GPU.

Torch provides the device memory (the workspace and the pressure vectors)
and the stream; every computation is a libcams call.
"""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _cams as C


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """Owns a libcams context, its workspace and the rock/well data of one
    problem.  `problem` is any object with the attributes of
    workloads.Problem (grid, fluid, rock, wells, options)."""

    def __init__(self, problem, device="cuda:0", stream=None, **overrides):
        self.pb = problem
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        g = C.cams_grid(problem.nx, problem.ny, problem.nz, problem.dx, problem.dy, problem.dz,
                        problem.rx, problem.ry, problem.rz)
        f = C.cams_fluid(problem.rho0, problem.c, problem.p0, problem.mu, problem.dt)
        o = C.cams_options(overrides.get("restriction", problem.restriction),
                           overrides.get("n_pre", problem.n_pre), overrides.get("n_post", problem.n_post),
                           overrides.get("precision", problem.precision),
                           overrides.get("smoother", getattr(problem, "smoother", C.CAMS_SMOOTH_BLOCK_ILU0)),
                           overrides.get("lin_rtol", problem.lin_rtol),
                           overrides.get("lin_maxit", problem.lin_maxit),
                           overrides.get("newton_tol", problem.newton_tol),
                           overrides.get("newton_maxit", problem.newton_maxit),
                           overrides.get("lin_atol", getattr(problem, "lin_atol", 0.0)),
                           overrides.get("basis_type", getattr(problem, "basis_type", 0)),
                           overrides.get("basis_tol", getattr(problem, "basis_tol", 0.0)),
                           overrides.get("coarse_tol", getattr(problem, "coarse_tol", 0.0)))
        self.options = o
        h = ctypes.c_void_p()
        C.check(C.cams_create(ctypes.byref(g), ctypes.byref(f), ctypes.byref(o),
                              ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)), None, "cams_create")
        self.ctx = h
        nbytes = C.cams_workspace_bytes(self.ctx)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        C.check(C.cams_set_workspace(self.ctx, ctypes.c_void_p(self._ws_ptr), nbytes), self.ctx,
                "cams_set_workspace")
        self.N = problem.n
        self.Nc = int(C.cams_num_coarse(self.ctx))
        perm = torch.as_tensor(np.ascontiguousarray(problem.perm, dtype=np.float64), device=self.device)
        phi = torch.as_tensor(np.ascontiguousarray(problem.phi, dtype=np.float64), device=self.device)
        q = None
        if problem.q is not None:
            q = torch.as_tensor(np.ascontiguousarray(problem.q, dtype=np.float64), device=self.device)
        self._rock = (perm, phi, q)
        self.reset_rock()
        for side, face in (("W", 0), ("E", 1)):
            bc = getattr(problem, "face_bc", None) or {}
            if side in bc:
                C.check(C.cams_set_face_dirichlet(self.ctx, face, float(bc[side])), self.ctx,
                        "cams_set_face_dirichlet")
        cells = np.array([w[0] for w in problem.wells], dtype=np.int64)
        vals = np.array([w[1] for w in problem.wells], dtype=np.float64)
        C.check(C.cams_set_wells(self.ctx, cells.ctypes.data_as(ctypes.c_void_p),
                                 vals.ctypes.data_as(ctypes.c_void_p), len(problem.wells)),
                self.ctx, "cams_set_wells")
        self.last_stats = C.cams_stats()

    def reset_rock(self):
        """(Re)load permeability and porosity: recomputes the transmissibilities
        and invalidates the basis, so the next step rebuilds it."""
        perm, phi, q = self._rock
        C.check(C.cams_set_rock(self.ctx, _ptr(perm), _ptr(phi), _ptr(q) if q is not None else None),
                self.ctx, "cams_set_rock")

    def coarse_solve(self, rc: torch.Tensor) -> torch.Tensor:
        """A_c^-1 rc with the current coarse factorisation (test hook)."""
        xc = torch.empty_like(rc)
        C.check(C.cams_debug_coarse_solve(self.ctx, _ptr(rc), _ptr(xc)), self.ctx, "cams_debug_coarse_solve")
        return xc

    def invalidate_basis(self):
        """The next step rebuilds the basis from the current transmissibilities."""
        C.check(C.cams_invalidate_basis(self.ctx), self.ctx, "cams_invalidate_basis")

    # ---- the five hot-path calls
    def assemble(self, p: torch.Tensor, pn: torch.Tensor) -> float:
        e = ctypes.c_double()
        C.check(C.cams_assemble(self.ctx, _ptr(p), _ptr(pn), ctypes.byref(e)), self.ctx, "cams_assemble")
        return e.value

    def build_basis(self):
        C.check(C.cams_build_basis(self.ctx), self.ctx, "cams_build_basis")

    def coarse_op(self):
        C.check(C.cams_coarse_op(self.ctx), self.ctx, "cams_coarse_op")

    def iterate(self, p: torch.Tensor) -> dict:
        st = C.cams_stats()
        C.check(C.cams_iterate(self.ctx, _ptr(p), ctypes.byref(st)), self.ctx, "cams_iterate")
        return st.as_dict()

    def newton_step(self, pn: torch.Tensor, p: torch.Tensor, check=True) -> dict:
        st = C.cams_stats()
        status = C.cams_newton_step(self.ctx, _ptr(pn), _ptr(p), ctypes.byref(st))
        self.last_stats = st
        if check:
            C.check(status, self.ctx, "cams_newton_step")
        d = st.as_dict()
        d["status"] = status
        return d

    def conservative_sweep(self, pn: torch.Tensor, p: torch.Tensor) -> torch.Tensor:
        """One MSFV stage at p (updated in place); returns the (3, N) two-point
        mass fluxes of that linear system at the new pressure."""
        flux = torch.empty((3, self.N), dtype=torch.float64, device=self.device)
        C.check(C.cams_conservative_sweep(self.ctx, _ptr(pn), _ptr(p), _ptr(flux)), self.ctx,
                "cams_conservative_sweep")
        return flux

    def newton_history(self, pn: torch.Tensor, p: torch.Tensor, cap=20000, check=True):
        """One time step with the norm history of every C-AMS iteration:
        (stats dict, Newton index (n,), ||r||_2 (n,), ||eps||_2 (n,))."""
        res = np.zeros(cap)
        err = np.zeros(cap)
        nwt = np.zeros(cap, dtype=np.int32)
        cnt = ctypes.c_int32()
        st = C.cams_stats()
        status = C.cams_newton_history(self.ctx, _ptr(pn), _ptr(p), res.ctypes.data_as(ctypes.c_void_p),
                                       err.ctypes.data_as(ctypes.c_void_p), nwt.ctypes.data_as(ctypes.c_void_p),
                                       cap, ctypes.byref(cnt), ctypes.byref(st))
        if check:
            C.check(status, self.ctx, "cams_newton_history")
        n = min(cnt.value, cap)
        d = st.as_dict()
        d["status"] = status
        d["entries"] = cnt.value
        return d, nwt[:n], res[:n], err[:n]

    def smooth_apply(self, z: torch.Tensor) -> torch.Tensor:
        x = torch.empty_like(z)
        C.check(C.cams_smooth_apply(self.ctx, _ptr(z), _ptr(x)), self.ctx, "cams_smooth_apply")
        return x

    # ---- learned basis
    def num_full_blocks(self) -> int:
        return int(C.cams_cnn_num_blocks(self.ctx))

    def cnn_patches(self, with_targets=True):
        """(features (B,3,729), targets (B,8,343) or None) of the full dual blocks;
        targets need a built (exact) basis."""
        nb = self.num_full_blocks()
        feat = torch.empty((nb, 3, 729), dtype=torch.float32, device=self.device)
        tgt = torch.empty((nb, 8, 343), dtype=torch.float32, device=self.device) if with_targets else None
        C.check(C.cams_cnn_patches(self.ctx, _ptr(feat), _ptr(tgt) if tgt is not None else None), self.ctx,
                "cams_cnn_patches")
        return feat, tgt

    def set_learned(self, params, fallback_tol=1e-2, guard_iters=0):
        """Use the network for full-block interiors (params: float32 device
        tensor), or exact local solves again (params None).  guard_iters > 0:
        the exact basis' C-AMS iterations per solve, for the global check
        (cams_set_learned_guard)."""
        C.check(C.cams_set_learned_guard(self.ctx, int(guard_iters)), self.ctx, "cams_set_learned_guard")
        if params is None:
            C.check(C.cams_set_learned(self.ctx, None, None, 0, 0.0), self.ctx, "cams_set_learned")
            self._learned = None
            return
        nbytes = C.cams_learned_scratch_bytes(self.ctx)
        scratch = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = (scratch.data_ptr() + 255) // 256 * 256
        C.check(C.cams_set_learned(self.ctx, _ptr(params), ctypes.c_void_p(ptr), nbytes, float(fallback_tol)),
                self.ctx, "cams_set_learned")
        self._learned = (params, scratch)

    def basis_stats(self) -> dict:
        a, b = ctypes.c_int32(), ctypes.c_int32()
        C.check(C.cams_basis_stats(self.ctx, ctypes.byref(a), ctypes.byref(b)), self.ctx, "cams_basis_stats")
        return {"learned_blocks": a.value, "fallback_blocks": b.value}

    def block_ratios(self) -> np.ndarray:
        """Local-equation ratio of the network's prediction per full dual
        block, from the last learned basis build (before fallback)."""
        n = self.num_full_blocks()
        out = np.zeros(n, dtype=np.float64)
        C.check(C.cams_basis_block_ratios(self.ctx, out.ctypes.data_as(ctypes.c_void_p), n), self.ctx,
                "cams_basis_block_ratios")
        return out

    # ---- measurement
    def profile(self, kernel=C.CAMS_PROF_SMOOTH_STEP):
        C.check(C.cams_profile(self.ctx, kernel), self.ctx, "cams_profile")

    def profile_read(self) -> dict:
        ms, n, b = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        C.check(C.cams_profile_read(self.ctx, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b)), self.ctx,
                "cams_profile_read")
        return {"total_ms": ms.value, "launches": n.value, "bytes": b.value}

    # ---- inspection
    def export(self, which: int) -> torch.Tensor:
        nbytes = C.cams_array_bytes(self.ctx, which)
        out = torch.empty(nbytes // 8, dtype=torch.float64, device=self.device)
        C.check(C.cams_export(self.ctx, which, _ptr(out), nbytes), self.ctx, "cams_export")
        return out

    def import_basis(self, P: torch.Tensor):
        """Use a saved basis (8*N float64 on this device, as export(CAMS_ARR_P)
        returns it) instead of rebuilding it (types B3/B4)."""
        P = P.to(device=self.device, dtype=torch.float64).contiguous()
        C.check(C.cams_import_basis(self.ctx, _ptr(P), P.numel() * 8), self.ctx, "cams_import_basis")

    def new_pressure(self) -> torch.Tensor:
        return torch.as_tensor(self.pb.initial_pressure(), dtype=torch.float64, device=self.device)

    def close(self):
        if self.ctx:
            C.cams_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
