"""Problem definitions for the compressible single-phase pressure solve.

A Problem holds everything the paper's problem statement needs (Sec. 2,
Eqs. (1)-(6); Sec. 4): the Cartesian grid and its coarsening ratio, the rock
(permeability, porosity), the fluid (density law, viscosity), the time step,
the Dirichlet (well) cells and the solver options.  Values are drawn from
seeded generators only; no solver arithmetic happens here.

Workloads:
  config1      2D 20x20, coarsening 4x4, ln k sigma 2, one time step (MSFV).
  config2      3D 64x64x32, coarsening 8^3, ln k sigma 3, 10 time steps (MSFE).
  config4      3D 256x256x128 channelised field, coarsening 8^3, 5 time steps.
  config5_eval 3D 128^3, coarsening 8, sigma 3 (learned-basis evaluation grid).
  batch_problems  uneven 3D instances for the batched solve.
  small_problem   tiny grids for oracle pins and quick parity tests.
"""

from __future__ import annotations

import dataclasses
from typing import List, Optional, Tuple

import numpy as np

from .fields import lognormal_permeability, channel_permeability

FV = 0  # restriction: finite-volume block sums
FE = 1  # restriction: transpose of prolongation

FP64 = 0
MIXED_FP32 = 1
MIXED_BF16 = 2

SMOOTH_BLOCK = 0      # block-Jacobi ILU(0) on 8x8x8 blocks
SMOOTH_REDBLACK = 1   # ILU(0) in red-black order
SMOOTH_BLOCK_ALT = 2  # block ILU(0), every other step on the half-block-shifted block grid
SMOOTH_NATURAL = 3    # ILU(0) of the whole matrix in natural (cell) order


@dataclasses.dataclass
class Problem:
    name: str
    nx: int
    ny: int
    nz: int
    rx: int
    ry: int
    rz: int
    perm: np.ndarray            # (N,) float64, cell permeability (isotropic)
    phi: np.ndarray             # (N,) float64, porosity
    wells: List[Tuple[int, float]]  # (cell index, fixed pressure)
    dx: float = 1.0
    dy: float = 1.0
    dz: float = 1.0
    rho0: float = 1.0
    c: float = 0.1
    p0: float = 0.0
    mu: float = 1.0
    dt: float = 0.1
    q: Optional[np.ndarray] = None  # (N,) source per unit volume, or None
    face_bc: Optional[dict] = None  # Dirichlet boundary faces {"W": p, "E": p} (x = 0 / x = nx-1 faces)
    n_steps: int = 1
    restriction: int = FE
    n_pre: int = 0
    n_post: int = 5
    lin_rtol: float = 1e-8
    lin_atol: float = 0.0           # absolute linear tolerance (0: relative only)
    lin_maxit: int = 500
    newton_tol: float = 1e-8
    newton_maxit: int = 30
    precision: int = FP64
    smoother: int = SMOOTH_BLOCK_ALT
    basis_type: int = 0             # 0 = B4, 1 = B1, 2 = B2, 3 = B3 (Sec. 3)
    basis_tol: float = 0.0          # B1/B2 adaptive update threshold (0: rebuild every Newton iteration)
    coarse_tol: float = 0.0         # adaptive coarse factorisation threshold (0: every Newton iteration)

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    def cell(self, i, j, k=0) -> int:
        return i + self.nx * (j + self.ny * k)

    def initial_pressure(self) -> np.ndarray:
        """Zero everywhere except at the Dirichlet cells (Sec. 4.1.3)."""
        p = np.zeros(self.n)
        for c, v in self.wells:
            p[c] = v
        return p

    def dirichlet_mask(self) -> np.ndarray:
        m = np.zeros(self.n, dtype=np.uint8)
        for c, _ in self.wells:
            m[c] = 1
        return m

    def with_options(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


def _column_wells(nx, ny, nz, ij_values):
    wells = []
    for (i, j), v in ij_values:
        for k in range(nz):
            wells.append((i + nx * (j + ny * k), float(v)))
    return wells


def config1() -> Problem:
    """2D 20x20, coarsening 4x4, ln k ~ N(0, 2^2) with correlation length 4,
    porosity 0.2, c = 0.1, dt = 0.1, injector p=1 at (0,0), producer p=0 at
    (19,19), one time step, MSFV restriction, 5 pre- and 5 post-smoothing."""
    nx, ny = 20, 20
    perm = lognormal_permeability((ny, nx), 0.0, 2.0, 4.0, seed=1).reshape(-1)
    phi = np.full(nx * ny, 0.2)
    wells = [(0, 1.0), (nx * ny - 1, 0.0)]
    return Problem("config1_2d_20x20", nx, ny, 1, 4, 4, 1, perm, phi, wells,
                   c=0.1, dt=0.1, n_steps=1, restriction=FV, n_pre=5, n_post=5)


def config2(precision: int = FP64) -> Problem:
    """3D 64x64x32, coarsening 8^3, ln k sigma 3 with correlation lengths
    (8,8,2), porosity U[0.1,0.3] per cell, c = 0.05, 10 steps of dt = 0.05,
    corner column wells p=1 at (0,0,:) and p=0 at (63,63,:), MSFE."""
    nx, ny, nz = 64, 64, 32
    perm = lognormal_permeability((nz, ny, nx), 0.0, 3.0, (2.0, 8.0, 8.0), seed=2).reshape(-1)
    rng = np.random.default_rng(20002)
    phi = rng.uniform(0.1, 0.3, size=nx * ny * nz)
    wells = _column_wells(nx, ny, nz, [((0, 0), 1.0), ((nx - 1, ny - 1), 0.0)])
    return Problem("config2_64x64x32", nx, ny, nz, 8, 8, 8, perm, phi, wells,
                   c=0.05, dt=0.05, n_steps=10, restriction=FE, n_pre=0, n_post=5,
                   precision=precision)


def config4(precision: int = MIXED_BF16) -> Problem:
    """3D 256x256x128 binary channelised field (k=1 channels, 1e-4 matrix,
    30% channel fraction), coarsening 8^3, porosity 0.2, c = 0.1, 5 steps of
    dt = 0.05, corner column wells."""
    nx, ny, nz = 256, 256, 128
    perm = channel_permeability((nz, ny, nx), seed=4).reshape(-1)
    phi = np.full(nx * ny * nz, 0.2)
    wells = _column_wells(nx, ny, nz, [((0, 0), 1.0), ((nx - 1, ny - 1), 0.0)])
    return Problem("config4_256x256x128_channel", nx, ny, nz, 8, 8, 8, perm, phi, wells,
                   c=0.1, dt=0.05, n_steps=5, restriction=FE, n_pre=0, n_post=5,
                   precision=precision)


def config5_eval(precision: int = MIXED_FP32) -> Problem:
    """3D 128^3, coarsening 8, ln k sigma 3, correlation length 8, c = 0.1,
    porosity 0.2, dt = 0.1, one time step."""
    n = 128
    perm = lognormal_permeability((n, n, n), 0.0, 3.0, 8.0, seed=5).reshape(-1)
    phi = np.full(n ** 3, 0.2)
    wells = _column_wells(n, n, n, [((0, 0), 1.0), ((n - 1, n - 1), 0.0)])
    return Problem("config5_eval_128^3", n, n, n, 8, 8, 8, perm, phi, wells,
                   c=0.1, dt=0.1, n_steps=1, restriction=FE, n_pre=0, n_post=5,
                   precision=precision)


def stretched_problem(alpha: float, seed: int = 8, n: int = 64, precision: int = FP64) -> Problem:
    """Test case 2 of Sec. 4.2 on a synthetic field: 64^3 cells of aspect
    ratio dx / alpha = dy = dz = 1, ln k lognormal sigma 2 (variance 4, the
    paper's permeability set 1) with correlation length 8 cells, Dirichlet
    line sources along the vertical columns (0, 0, :) p = 1 and
    (63, 63, :) p = 0; coarsening 8x8x8 for alpha = 1 and 2x8x8 for the
    stretched grids (the paper's choice); c = 0.1, porosity 0.2, dt = 0.1,
    one time step, MSFE."""
    perm = lognormal_permeability((n, n, n), 0.0, 2.0, 8.0, seed=seed).reshape(-1)
    r = (8, 8, 8) if alpha == 1 else (2, 8, 8)
    wells = _column_wells(n, n, n, [((0, 0), 1.0), ((n - 1, n - 1), 0.0)])
    return Problem(f"stretched_alpha{alpha:g}_{n}^3", n, n, n, *r, perm, np.full(n ** 3, 0.2), wells,
                   dx=float(alpha), c=0.1, dt=0.1, n_steps=1, restriction=FE, n_pre=0, n_post=5,
                   precision=precision)


def variance_problem(sigma: float, seed: int, layered: bool = False, n: int = 64, restriction: int = FE,
                     precision: int = FP64) -> Problem:
    """Test case 3 of Sec. 4.2 on synthetic fields: 64^3, ln k lognormal with
    standard deviation sigma (2, 4 or 8), patchy (correlation length 8
    cells) or layered (16 x 16 cells in x-y, 1 cell in z); the default
    boundary conditions of the paper's test cases: pressure 1 on the west
    face, 0 on the east face, no flow elsewhere, no wells; coarsening 8^3,
    c = 0.1, porosity 0.2, dt = 0.1, one time step."""
    corr = (1.0, 16.0, 16.0) if layered else 8.0
    perm = lognormal_permeability((n, n, n), 0.0, sigma, corr, seed=seed).reshape(-1)
    kind = "layered" if layered else "patchy"
    return Problem(f"variance_{kind}_sigma{sigma:g}_s{seed}", n, n, n, 8, 8, 8, perm, np.full(n ** 3, 0.2), [],
                   c=0.1, dt=0.1, n_steps=1, restriction=restriction, n_pre=0, n_post=5, precision=precision,
                   face_bc={"W": 1.0, "E": 0.0})


def small_problem(nx, ny, nz, r, seed=7, sigma=1.5, corr=3.0, c=0.1, dt=0.1,
                  restriction=FE, n_pre=0, n_post=5, wells="corners",
                  phi_range=(0.1, 0.3)) -> Problem:
    """Tiny/medium grids for pins and parity tests.  r: int or (rx, ry, rz)."""
    if np.isscalar(r):
        rx = ry = int(r)
        rz = int(r) if nz > 1 else 1
    else:
        rx, ry, rz = (int(v) for v in r)
    shape = (nz, ny, nx) if nz > 1 else (ny, nx)
    perm = lognormal_permeability(shape, 0.0, sigma, corr, seed=seed).reshape(-1)
    rng = np.random.default_rng(seed + 100000)
    phi = rng.uniform(phi_range[0], phi_range[1], size=nx * ny * nz)
    if wells == "corners":
        w = _column_wells(nx, ny, nz, [((0, 0), 1.0), ((nx - 1, ny - 1), 0.0)])
    elif wells == "none":
        w = []
    else:
        w = list(wells)
    return Problem(f"small_{nx}x{ny}x{nz}_r{rx}{ry}{rz}_s{seed}", nx, ny, nz, rx, ry, rz,
                   perm, phi, w, c=c, dt=dt, restriction=restriction,
                   n_pre=n_pre, n_post=n_post)


def batch_problems(count=256, seed=3, precision=MIXED_FP32) -> List[Problem]:
    """Uneven 3D instances: nx, ny ~ U{32..96}, nz ~ U{16..48}, coarsening per
    axis ~ U{4..8}, ln k sigma ~ U[1,4] (correlation 8x8x2), c ~ U[0.01,0.2],
    porosity 0.2, dt 0.05, corner column wells, one Newton iteration each."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        nx = int(rng.integers(32, 97))
        ny = int(rng.integers(32, 97))
        nz = int(rng.integers(16, 49))
        rx, ry, rz = (int(v) for v in rng.integers(4, 9, size=3))
        sigma = float(rng.uniform(1.0, 4.0))
        c = float(rng.uniform(0.01, 0.2))
        perm = lognormal_permeability((nz, ny, nx), 0.0, sigma, (2.0, 8.0, 8.0),
                                      seed=int(seed * 100000 + b)).reshape(-1)
        phi = np.full(nx * ny * nz, 0.2)
        wells = _column_wells(nx, ny, nz, [((0, 0), 1.0), ((nx - 1, ny - 1), 0.0)])
        out.append(Problem(f"batch{b}_{nx}x{ny}x{nz}_r{rx}{ry}{rz}", nx, ny, nz, rx, ry, rz,
                           perm, phi, wells, c=c, dt=0.05, n_steps=1, restriction=FE,
                           n_pre=0, n_post=5, precision=precision, newton_maxit=1))
    return out
