"""Pins of the CPU oracle against the paper and against mathematics.

Each test checks the oracle against something other than itself: closed
forms (homogeneous media, 1D series resistances), invariants (partition of
unity, conservation, symmetry), library routines (SciPy sparse LU, NumPy
dense solves, SciPy triangular solves) and brute force on tiny grids.
"""

from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from tests import helpers
from workloads import Problem, config1, small_problem
from workloads.configs import FE, FV


def homogeneous(nx, ny, nz, r, k=2.5, dx=1.0, dy=1.0, dz=1.0, wells="corners", c=0.1):
    pb = small_problem(nx, ny, nz, r, wells=wells, c=c)
    pb.perm = np.full(pb.n, k)
    pb.dx, pb.dy, pb.dz = dx, dy, dz
    return pb


# ---------------------------------------------------------------- TPFA ----

def test_tpfa_homogeneous_closed_form():
    pb = homogeneous(5, 4, 3, 2, k=3.0, dx=2.0, dy=0.5, dz=1.5)
    T = oracle.transmissibility(pb)
    Tx, Ty, Tz = (t.reshape(3, 4, 5) for t in T)
    # interior faces: k * area / spacing; boundary faces: no flow
    assert np.allclose(Tx[:, :, :-1], 3.0 * 0.5 * 1.5 / 2.0, rtol=1e-15)
    assert np.allclose(Ty[:, :-1, :], 3.0 * 2.0 * 1.5 / 0.5, rtol=1e-15)
    assert np.allclose(Tz[:-1, :, :], 3.0 * 2.0 * 0.5 / 1.5, rtol=1e-15)
    assert np.all(Tx[:, :, -1] == 0) and np.all(Ty[:, -1, :] == 0) and np.all(Tz[-1] == 0)


def test_tpfa_series_resistance_steady_1d():
    """Steady incompressible flow through a 1D chain of cells: the pressure
    at each cell centre falls in proportion to the accumulated half-cell
    resistances h / (2 k A) (textbook layered-medium result)."""
    n = 9
    rng = np.random.default_rng(0)
    k = np.exp(rng.normal(0, 1.5, n))
    pb = Problem("chain", n, 2, 1, 3, 2, 1, np.repeat(k[None, :], 2, axis=0).ravel(),
                 np.full(2 * n, 0.2), [(0, 1.0), (n, 1.0), (n - 1, 0.0), (2 * n - 1, 0.0)],
                 dx=1.3, dy=0.7, c=0.0, dt=1.0)
    T = oracle.transmissibility(pb)
    p0 = pb.initial_pressure()
    p, _ = helpers.direct_newton(pb, T, p0, p0)
    area = pb.dy * pb.dz
    half = (pb.dx / 2) / (k * area)          # half-cell resistance
    # resistance from centre of cell 0 to centre of cell m
    R = np.concatenate([[0.0], np.cumsum(half[:-1] + half[1:])])
    expected = 1.0 - R / R[-1]
    assert np.allclose(p[:n], expected, rtol=0, atol=1e-13)
    assert np.allclose(p[n:], expected, rtol=0, atol=1e-13)


# ------------------------------------------------------------ assembly ----

def test_jacobian_equals_finite_difference_at_uniform_state():
    """At a uniform state p = p^n the paper's linearisation (Eqs. (3)-(6))
    is the exact Jacobian of the residual of Eq. (2): the lagged face
    densities multiply zero pressure differences and c^nu uses rho^n."""
    pb = small_problem(6, 5, 4, 2, wells="none", c=0.3, dt=0.2)
    T = oracle.transmissibility(pb)
    p = np.full(pb.n, 0.37)
    W, diag, r, _ = oracle.linear_system(pb, T, p, p)
    A = helpers.stencil_matrix(pb, W, diag).toarray()
    h = 1e-6
    J = np.zeros((pb.n, pb.n))
    for j in range(pb.n):
        e = np.zeros(pb.n); e[j] = h
        Fp, _ = oracle.nonlinear_residual(pb, T, p + e, p)
        Fm, _ = oracle.nonlinear_residual(pb, T, p - e, p)
        J[:, j] = (Fp - Fm) / (2 * h)
    assert np.max(np.abs(J - A)) <= 1e-7 * np.max(np.abs(A))
    assert np.max(np.abs(r)) == 0.0


def test_incompressible_residual_is_affine():
    """c = 0: the residual is affine in p with the assembled matrix as its
    exact Jacobian (no density lag), so F(p+x) - F(p) = A x."""
    pb = small_problem(7, 6, 3, 3, c=0.0)
    T = oracle.transmissibility(pb)
    rng = np.random.default_rng(1)
    p = pb.initial_pressure() + 0.0
    p[pb.dirichlet_mask() == 0] = rng.uniform(0, 1, (pb.dirichlet_mask() == 0).sum())
    x = rng.normal(size=pb.n)
    x[pb.dirichlet_mask() == 1] = 0.0
    W, diag, r, _ = oracle.linear_system(pb, T, p, p)
    F1, _ = oracle.nonlinear_residual(pb, T, p, p)
    F2, _ = oracle.nonlinear_residual(pb, T, p + x, p)
    Ax = helpers.stencil_matrix(pb, W, diag) @ x
    free = pb.dirichlet_mask() == 0
    assert np.allclose((F2 - F1)[free], Ax[free], rtol=0, atol=1e-12 * np.abs(Ax).max())


def test_fluxes_conserve_mass():
    """Closed domain, no wells: summing Eq. (2) over all cells, inter-cell
    fluxes cancel, so dt * sum_i F_i does not depend on dt."""
    pb = small_problem(6, 6, 4, 2, wells="none", c=0.2)
    T = oracle.transmissibility(pb)
    rng = np.random.default_rng(2)
    p = rng.uniform(0, 1, pb.n)
    pn = rng.uniform(0, 1, pb.n)
    s = []
    for dt in (0.1, 0.7):
        pb.dt = dt
        F, _ = oracle.nonlinear_residual(pb, T, p, pn)
        s.append(dt * F.sum())
    assert abs(s[0] - s[1]) <= 1e-12 * abs(s[0])


def test_matrix_is_symmetric_m_matrix():
    pb = config1()
    T = oracle.transmissibility(pb)
    p = np.random.default_rng(3).uniform(0, 1, pb.n)
    W, diag, r, _ = oracle.linear_system(pb, T, p, pb.initial_pressure())
    A = helpers.stencil_matrix(pb, W, diag)
    assert abs(A - A.T).max() == 0
    off = A - sp.diags(A.diagonal())
    assert off.max() <= 0
    rowsum = np.asarray(A.sum(axis=1)).ravel()
    assert np.all(rowsum > 0)          # accumulation makes rows strictly dominant
    dm = pb.dirichlet_mask() == 1
    assert np.all(r[dm] == 0) and np.all(diag[dm] == 1)


def test_incompressible_newton_converges_in_one_iteration():
    pb = small_problem(8, 8, 4, 4, c=0.0)
    T = oracle.transmissibility(pb)
    P = oracle.basis_b4(pb, T)
    p0 = pb.initial_pressure()
    p, rc, st = oracle.newton_step(pb, T, P, p0, p0, lin_rtol=1e-12, newton_tol=1e-10)
    assert rc == 0 and st["newton_iters"] == 1


def test_converged_state_balances_well_inflow():
    """At convergence of a time step with no sources, the mass gained in the
    free cells equals the net inflow through faces adjacent to the
    Dirichlet cells (global balance of Eq. (1))."""
    pb = small_problem(10, 8, 4, 4, c=0.1)
    T = oracle.transmissibility(pb)
    P = oracle.basis_b4(pb, T)
    p0 = pb.initial_pressure()
    p, rc, st = oracle.newton_step(pb, T, P, p0, p0, lin_rtol=1e-13, newton_tol=1e-13)
    assert rc == 0
    rho = pb.rho0 * np.exp(pb.c * (p - pb.p0))
    rho_n = pb.rho0 * np.exp(pb.c * (p0 - pb.p0))
    dm = pb.dirichlet_mask() == 1
    gained = (pb.phi * (rho - rho_n) / pb.dt)[~dm].sum()
    # inflow through faces between a Dirichlet and a free cell
    nx, ny, nz = pb.nx, pb.ny, pb.nz
    inflow = 0.0
    for a in range(pb.n):
        i, j, k = a % nx, (a // nx) % ny, a // (nx * ny)
        for (di, dj, dk, Tf) in ((1, 0, 0, T[0]), (0, 1, 0, T[1]), (0, 0, 1, T[2])):
            if i + di >= nx or j + dj >= ny or k + dk >= nz:
                continue
            b = a + di + nx * (dj + ny * dk)
            if dm[a] == dm[b]:
                continue
            d, f = (a, b) if dm[a] else (b, a)
            inflow += Tf[a] * 0.5 * (rho[a] + rho[b]) * (p[d] - p[f])
    assert abs(gained - inflow) <= 1e-9 * abs(inflow)


# -------------------------------------------------------- coarse grids ----

def test_vertex_placement_and_levels_brute_force():
    assert list(oracle.vertex_coords(20, 4)) == [2, 6, 10, 14, 18]
    assert list(oracle.vertex_coords(64, 8)) == [4 + 8 * a for a in range(8)]
    assert list(oracle.vertex_coords(10, 4)) == [2, 6, 9]        # last block has length 2
    pb = small_problem(10, 9, 7, (4, 3, 3))
    lv = oracle.cell_levels(pb).reshape(7, 9, 10)
    vx, vy, vz = (set(oracle.vertex_coords(n, r)) for n, r in ((10, 4), (9, 3), (7, 3)))
    for k in range(7):
        for j in range(9):
            for i in range(10):
                assert lv[k, j, i] == (i in vx) + (j in vy) + (k in vz)
    assert (lv == 3).sum() == len(vx) * len(vy) * len(vz)
    assert oracle.num_coarse(pb) == 3 * 3 * 3


# --------------------------------------------------------------- basis ----

def _hat(n, r):
    """Per-axis 1D hat weights (lower, upper) of the bracketing vertices."""
    v = list(oracle.vertex_coords(n, r))
    lo = np.zeros(n); hi = np.zeros(n)
    for x in range(n):
        a = max([b for b in range(len(v)) if v[b] <= x], default=0)
        if x < v[0] or x >= v[-1] or x == v[a]:
            lo[x], hi[x] = 1.0, 0.0
        else:
            t = (x - v[a]) / (v[a + 1] - v[a])
            lo[x], hi[x] = 1.0 - t, t
    return lo, hi


@pytest.mark.parametrize("shape,r,sp_", [((12, 9, 1), (4, 3, 1), (1.0, 1.0, 1.0)),
                                          ((10, 11, 9), (4, 4, 3), (1.0, 2.0, 0.5)),
                                          ((16, 16, 16), (8, 8, 8), (1.0, 1.0, 1.0))])
def test_basis_homogeneous_is_multilinear_hat(shape, r, sp_):
    nx, ny, nz = shape
    pb = homogeneous(nx, ny, nz, r, dx=sp_[0], dy=sp_[1], dz=sp_[2])
    T = oracle.transmissibility(pb)
    P = oracle.basis_b4(pb, T)
    hx, hy, hz = _hat(nx, pb.rx), _hat(ny, pb.ry), _hat(nz, pb.rz) if nz > 1 else (np.ones(1), np.zeros(1))
    for s in range(8):
        bx, by, bz = s & 1, (s >> 1) & 1, (s >> 2) & 1
        expect = (hz[bz][:, None, None] * hy[by][None, :, None] * hx[bx][None, None, :]).ravel()
        assert np.allclose(P[s], expect, rtol=0, atol=1e-13), s


def test_basis_edge_series_resistance():
    """Along a dual edge the B4 basis is the 1D harmonic interpolant:
    Phi_upper(m) = (sum of face resistances up to m) / (total resistance),
    computed here in exact rational arithmetic."""
    pb = small_problem(17, 9, 1, (8, 4, 1), sigma=2.0, seed=11)
    T = oracle.transmissibility(pb)
    P = oracle.basis_b4(pb, T)
    v = list(oracle.vertex_coords(17, 8))   # [4, 12, 16]
    j = list(oracle.vertex_coords(9, 4))[0]
    Tx = T[0].reshape(9, 17)[j]
    res = [Fraction(1) / Fraction(float(t)) if t > 0 else None for t in Tx]
    total = sum(res[v[0]:v[1]])
    for m in range(v[0] + 1, v[1]):
        up = sum(res[v[0]:m]) / total
        cell = m + 17 * j
        assert abs(P[1][cell] - float(up)) <= 1e-14
        assert abs(P[0][cell] - float(1 - up)) <= 1e-14


@pytest.mark.parametrize("shape,r", [((20, 20, 1), (4, 4, 1)), ((13, 11, 9), (4, 3, 3)),
                                      ((24, 16, 16), (8, 8, 8))])
def test_basis_partition_of_unity_and_bounds(shape, r):
    pb = small_problem(*shape, r, sigma=2.5, seed=5)
    T = oracle.transmissibility(pb)
    P = oracle.basis_b4(pb, T)
    assert np.max(np.abs(P.sum(axis=0) - 1.0)) <= 1e-12
    assert P.min() >= -1e-14 and P.max() <= 1 + 1e-12
    nodes = oracle.slot_nodes(pb)
    lv = oracle.cell_levels(pb)
    dim = 3 if pb.nz > 1 else 2
    vert = np.nonzero(lv == dim)[0]
    assert np.all(P[0][vert] == 1.0) and np.all(P[1:, vert] == 0.0)
    # weights only on existing nodes
    assert np.all(P[nodes < 0] == 0.0)
    # at most 2^dim nonzeros per row
    assert np.max((P != 0).sum(axis=0)) <= 2 ** dim


def test_basis_solves_the_local_problems():
    """Interior rows of the B4 basis satisfy T Phi = 0 exactly (Eq. (11))."""
    pb = small_problem(16, 16, 8, (8, 8, 4), sigma=2.0, seed=9)
    T = oracle.transmissibility(pb)
    P = oracle.basis_b4(pb, T)
    Nc = oracle.num_coarse(pb)
    Pm = helpers.prolongation_matrix(pb.with_options(wells=[]), P, oracle.slot_nodes(pb), Nc)
    Top = helpers.stencil_matrix(pb, T, np.zeros(pb.n))
    Top = Top - sp.diags(np.asarray(Top.sum(axis=1)).ravel())   # zero row sums
    res = (Top @ Pm).toarray()
    lv = oracle.cell_levels(pb)
    assert np.max(np.abs(res[lv == 0])) <= 1e-12 * np.abs(T).max()


# -------------------------------------------------- coarse operator ----

@pytest.mark.parametrize("restriction", [FV, FE])
def test_coarse_operator_equals_sparse_triple_product(restriction):
    pb = small_problem(16, 12, 8, (4, 4, 4), sigma=2.0)
    T = oracle.transmissibility(pb)
    P = oracle.basis_b4(pb, T)
    p = np.random.default_rng(4).uniform(0, 1, pb.n)
    W, diag, r, _ = oracle.linear_system(pb, T, p, pb.initial_pressure())
    Ac = oracle.coarse_operator(pb, W, diag, P, restriction)
    Nc = oracle.num_coarse(pb)
    A = helpers.stencil_matrix(pb, W, diag)
    Ph = helpers.prolongation_matrix(pb, P, oracle.slot_nodes(pb), Nc)
    R = Ph.T if restriction == FE else helpers.fv_restriction_matrix(oracle.primal_block(pb), Nc)
    ref = (R @ A @ Ph).toarray()
    assert np.max(np.abs(Ac - ref)) <= 1e-13 * np.abs(ref).max()
    if restriction == FE:
        assert np.max(np.abs(Ac - Ac.T)) <= 1e-15 * np.abs(Ac).max() * 10
        np.linalg.cholesky(Ac)      # SPD (Sec. 4.2: MSFE always converges)


def test_lu_solve_matches_numpy():
    rng = np.random.default_rng(5)
    A = rng.normal(size=(40, 40)) + 3 * np.eye(40)
    b = rng.normal(size=40)
    LU, piv = oracle.lu_factor(A)
    x = oracle.lu_solve(LU, piv, b)
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-13, atol=1e-13)


# ------------------------------------------------------------- ILU(0) ----

@pytest.mark.parametrize("ordering", ["natural", "redblack"])
def test_ilu0_defining_property_and_apply(ordering):
    """ILU(0): (L U)_ij = A_ij on the sparsity pattern of A (permuted), and
    one application equals forward/backward substitution with L, U."""
    pb = small_problem(7, 6, 5, 3, sigma=2.0)
    T = oracle.transmissibility(pb)
    p = np.random.default_rng(6).uniform(0, 1, pb.n)
    W, diag, r, _ = oracle.linear_system(pb, T, p, pb.initial_pressure())
    order = np.arange(pb.n) if ordering == "natural" else oracle.redblack_order(pb)
    ilu = oracle.ILU0(pb, W, diag, order=order)
    rp, col, val = ilu.export()
    N = pb.n
    F = sp.csr_matrix((val, col, rp), shape=(N, N)).toarray()
    L = np.tril(F, -1) + np.eye(N)
    U = np.triu(F)
    A = helpers.stencil_matrix(pb, W, diag).toarray()[np.ix_(order, order)]
    pattern = A != 0
    assert np.max(np.abs((L @ U - A)[pattern])) <= 1e-13 * np.abs(A).max()
    assert np.all(np.diag(U) > 0)            # M-matrix: positive pivots
    z = np.random.default_rng(7).normal(size=N)
    y = spla.spsolve_triangular(sp.csr_matrix(L), z[order], lower=True)
    x = spla.spsolve_triangular(sp.csr_matrix(U), y, lower=False)
    expect = np.zeros(N); expect[order] = x
    assert np.allclose(ilu.apply(z), expect, rtol=1e-12, atol=1e-14)


def test_natural_ilu0_of_a_chain_is_the_exact_factorisation():
    """A 1D chain of cells gives a tridiagonal matrix; natural-order ILU(0)
    drops no fill there, so it is the exact LU factorisation and one
    application of the smoother solves A x = z (to rounding)."""
    n = 23
    rng = np.random.default_rng(12)
    pb = Problem("chain", n, 1, 1, 3, 1, 1, np.exp(rng.normal(0, 1.5, n)), np.full(n, 0.2),
                 [(0, 1.0)], c=0.1, dt=0.5)
    T = oracle.transmissibility(pb)
    W, diag, _, _ = oracle.linear_system(pb, T, rng.uniform(0, 1, n), pb.initial_pressure())
    ilu = oracle.smoother_for(pb, W, diag, oracle.SMOOTH_NATURAL)
    A = helpers.stencil_matrix(pb, W, diag).toarray()
    z = rng.normal(size=n)
    x = ilu.apply(z)
    assert np.allclose(A @ x, z, rtol=0, atol=1e-13 * np.abs(z).max())


def test_natural_ilu0_is_the_diagonal_recurrence():
    """For a 7-point operator in natural order, ILU(0) changes only the
    diagonal: the pivots follow d_n = diag_n - sum over the lower neighbours
    m of W_mn^2 / d_m, and M^{-1} z is a forward sweep
    y_n = (z_n + sum_lower W y_m) / d_n followed by a backward sweep
    x_n = y_n + (sum_upper W x_m) / d_n.  Written out here cell by cell on a
    ragged 3D grid with well cells and compared with the oracle's generic
    (row-by-row elimination) factor."""
    pb = small_problem(9, 7, 5, 3, sigma=2.0)
    T = oracle.transmissibility(pb)
    rng = np.random.default_rng(13)
    W, diag, _, _ = oracle.linear_system(pb, T, rng.uniform(0, 1, pb.n), pb.initial_pressure())
    Wx, Wy, Wz = W
    N, nx, sxy = pb.n, pb.nx, pb.nx * pb.ny

    def lower(n):
        i, j, k = n % nx, (n // nx) % pb.ny, n // sxy
        return [(m, w[m]) for ok, m, w in ((i > 0, n - 1, Wx), (j > 0, n - nx, Wy), (k > 0, n - sxy, Wz)) if ok]

    def upper(n):
        i, j, k = n % nx, (n // nx) % pb.ny, n // sxy
        return [(m, w[n]) for ok, m, w in ((i + 1 < nx, n + 1, Wx), (j + 1 < pb.ny, n + nx, Wy),
                                           (k + 1 < pb.nz, n + sxy, Wz)) if ok]

    d = np.zeros(N)
    for n in range(N):
        d[n] = diag[n] - sum(w * w / d[m] for m, w in lower(n))
    z = rng.normal(size=N)
    y = np.zeros(N)
    for n in range(N):
        y[n] = (z[n] + sum(w * y[m] for m, w in lower(n))) / d[n]
    x = np.zeros(N)
    for n in reversed(range(N)):
        x[n] = y[n] + sum(w * x[m] for m, w in upper(n)) / d[n]
    ilu = oracle.smoother_for(pb, W, diag, oracle.SMOOTH_NATURAL)
    rp, col, val = ilu.export()
    F = sp.csr_matrix((val, col, rp), shape=(N, N))
    assert np.allclose(F.diagonal(), d, rtol=1e-13, atol=0)
    assert np.allclose(ilu.apply(z), x, rtol=1e-12, atol=1e-14)


# -------------------------------------------------------------- C-AMS ----

def _setup(pb, restriction):
    T = oracle.transmissibility(pb)
    P = oracle.basis_b4(pb, T)
    p = pb.initial_pressure()
    W, diag, r, _ = oracle.linear_system(pb, T, p, p)
    Ac = oracle.coarse_operator(pb, W, diag, P, restriction)
    LU, piv = oracle.lu_factor(Ac)
    return T, P, W, diag, r, LU, piv


def test_msfv_stage_is_conservative():
    """After the MSFV coarse stage the residual sums to zero over every
    primal block (Sec. 4: a conservative velocity can be built)."""
    pb = small_problem(16, 16, 8, (4, 4, 4), sigma=2.0)
    T, P, W, diag, r, LU, piv = _setup(pb, FV)
    dc = oracle.lu_solve(LU, piv, oracle.restrict(pb, P, FV, r))
    d1 = oracle.prolong(pb, P, dc)
    r1 = r - oracle.matvec(pb, W, diag, d1)
    blk = oracle.primal_block(pb)
    sums = np.bincount(blk, weights=r1)
    assert np.max(np.abs(sums)) <= 1e-12 * np.abs(r).sum()


def test_msfe_stage_is_galerkin_orthogonal():
    pb = small_problem(16, 16, 8, (4, 4, 4), sigma=2.0)
    T, P, W, diag, r, LU, piv = _setup(pb, FE)
    dc = oracle.lu_solve(LU, piv, oracle.restrict(pb, P, FE, r))
    d1 = oracle.prolong(pb, P, dc)
    r1 = r - oracle.matvec(pb, W, diag, d1)
    Nc = oracle.num_coarse(pb)
    Ph = helpers.prolongation_matrix(pb, P, oracle.slot_nodes(pb), Nc)
    assert np.max(np.abs(Ph.T @ r1)) <= 1e-12 * np.abs(r).sum()


@pytest.mark.parametrize("restriction,n_pre,smoother", [(FV, 0, "rb"), (FE, 0, "rb"), (FV, 5, "rb"),
                                                        (FE, 0, "alt"), (FV, 5, "alt")])
def test_cams_converges_to_sparse_lu_solution(restriction, n_pre, smoother):
    pb = small_problem(16, 16, 8, (4, 4, 4), sigma=2.0)
    T, P, W, diag, r, LU, piv = _setup(pb, restriction)
    ilu = oracle.ILU0(pb, W, diag) if smoother == "rb" else oracle.smoother_for(pb, W, diag, oracle.SMOOTH_BLOCK_ALT)
    d, its, hist = oracle.cams_solve(pb, W, diag, P, restriction, LU, piv, ilu, r,
                                     n_pre=n_pre, n_post=5, rtol=1e-14, maxit=300)
    assert its > 0
    ref = spla.splu(helpers.stencil_matrix(pb, W, diag).tocsc()).solve(r)
    assert np.max(np.abs(d - ref)) <= 1e-12 * np.abs(ref).max()
    # deterministic iteration count and iterates
    d2, its2, _ = oracle.cams_solve(pb, W, diag, P, restriction, LU, piv, ilu, r,
                                    n_pre=n_pre, n_post=5, rtol=1e-14, maxit=300)
    assert its2 == its and np.array_equal(d, d2)


@pytest.mark.parametrize("smoother", [None, oracle.SMOOTH_NATURAL, oracle.SMOOTH_REDBLACK])
def test_config1_newton_matches_direct_newton(smoother):
    """Converged C-AMS Newton (MSFV, 5 pre + 5 post ILU(0); the problem's
    block smoother, the natural-order global one or the red-black one)
    equals Newton with sparse LU solves (C-AMS is an exact solver, Sec. 1)."""
    pb = config1()
    T = oracle.transmissibility(pb)
    P = oracle.basis_b4(pb, T)
    p0 = pb.initial_pressure()
    p, rc, st = oracle.newton_step(pb, T, P, p0, p0, lin_rtol=1e-13, newton_tol=1e-12, smoother=smoother)
    assert rc == 0
    ref, _ = helpers.direct_newton(pb, T, p0, p0, tol=1e-12)
    assert np.max(np.abs(p - ref)) <= 1e-10 * np.abs(ref).max()


@pytest.mark.slow
def test_3d_newton_matches_direct_newton_fe():
    pb = small_problem(24, 24, 16, 8, sigma=3.0, c=0.05, dt=0.05)
    T = oracle.transmissibility(pb)
    P = oracle.basis_b4(pb, T)
    p0 = pb.initial_pressure()
    p, rc, st = oracle.newton_step(pb, T, P, p0, p0, restriction=FE, lin_rtol=1e-13, newton_tol=1e-12)
    assert rc == 0
    ref, _ = helpers.direct_newton(pb, T, p0, p0, tol=1e-12)
    assert np.max(np.abs(p - ref)) <= 1e-10 * np.abs(ref).max()


def test_block_ilu0_is_ilu0_of_the_block_diagonal_part():
    """Block-Jacobi ILU(0): the factor reproduces, on its sparsity pattern,
    the matrix with couplings across 8x8x8 block faces removed (built here
    from geometry), and has no entry coupling two blocks."""
    pb = small_problem(19, 17, 11, 4, sigma=2.0)
    T = oracle.transmissibility(pb)
    p = np.random.default_rng(8).uniform(0, 1, pb.n)
    W, diag, r, _ = oracle.linear_system(pb, T, p, pb.initial_pressure())
    ilu = oracle.ILU0(pb, W, diag, block=(8, 8, 8))
    rp, col, val = ilu.export()
    N = pb.n
    F = sp.csr_matrix((val, col, rp), shape=(N, N)).toarray()
    L = np.tril(F, -1) + np.eye(N)
    U = np.triu(F)
    A = helpers.stencil_matrix(pb, W, diag).toarray()
    idx = np.arange(N)
    i, j, k = idx % pb.nx, (idx // pb.nx) % pb.ny, idx // (pb.nx * pb.ny)
    blk = (i // 8) + 100 * (j // 8) + 10000 * (k // 8)
    same = blk[:, None] == blk[None, :]
    Ab = np.where(same, A, 0.0)
    pattern = Ab != 0
    assert np.max(np.abs((L @ U - Ab)[pattern])) <= 1e-13 * np.abs(A).max()
    assert np.all(F[~same] == 0)
    z = np.random.default_rng(9).normal(size=N)
    x = np.linalg.solve(U, np.linalg.solve(L, z))
    assert np.allclose(ilu.apply(z), x, rtol=1e-11, atol=1e-13)


def _factor_dense(ilu, N):
    rp, col, val = ilu.export()
    return sp.csr_matrix((val, col, rp), shape=(N, N)).toarray()


def test_shifted_block_grid_cuts():
    """The shifted block grid cuts the axes where the cyclic positions
    (cell + offset) mod n cross a multiple of the block size.  Worked by hand
    for blocks of 4 cells: x (10 cells, offset 2) is cut after cells 1, 5
    and 7 (blocks {8, 9, 0, 1}, {2..5}, {6, 7}); y (6 cells, offset 1) after
    cells 2 and 4 (blocks {5, 0, 1, 2}, {3, 4})."""
    pb = small_problem(10, 6, 1, (2, 2, 1), sigma=1.0, wells="none")
    T = oracle.transmissibility(pb)
    p = np.random.default_rng(11).uniform(0, 1, pb.n)
    W, diag, r, _ = oracle.linear_system(pb, T, p, pb.initial_pressure())
    F = _factor_dense(oracle.ILU0(pb, W, diag, block=(4, 4, 1), shift=(2, 1, 0)), pb.n)
    nx, ny = pb.nx, pb.ny
    for j in range(ny):
        for i in range(nx - 1):
            a, b = i + nx * j, i + 1 + nx * j
            assert (F[b, a] != 0) == (i not in (1, 5, 7)), (i, j)
            assert (F[a, b] != 0) == (i not in (1, 5, 7)), (i, j)
    for j in range(ny - 1):
        for i in range(nx):
            a, b = i + nx * j, i + nx * (j + 1)
            assert (F[b, a] != 0) == (j not in (2, 4)), (i, j)


def test_shifted_block_ilu0_is_ilu0_of_the_block_diagonal_part():
    """The shifted block-Jacobi ILU(0) on a ragged grid: block labels made
    here by rolling the unshifted labels of each axis; the factor reproduces
    the block-diagonal part of A on its pattern, couples no two blocks, and
    one application equals the triangular solves."""
    pb = small_problem(19, 17, 11, 4, sigma=2.0)
    T = oracle.transmissibility(pb)
    p = np.random.default_rng(12).uniform(0, 1, pb.n)
    W, diag, r, _ = oracle.linear_system(pb, T, p, pb.initial_pressure())
    ilu = oracle.ILU0(pb, W, diag, block=(8, 8, 8), shift=(4, 4, 4))
    N = pb.n
    F = _factor_dense(ilu, N)
    L = np.tril(F, -1) + np.eye(N)
    U = np.triu(F)
    A = helpers.stencil_matrix(pb, W, diag).toarray()
    lab = [np.roll(np.arange(n) // 8, -4) for n in (pb.nx, pb.ny, pb.nz)]
    idx = np.arange(N)
    i, j, k = idx % pb.nx, (idx // pb.nx) % pb.ny, idx // (pb.nx * pb.ny)
    blk = lab[0][i] + 100 * lab[1][j] + 10000 * lab[2][k]
    same = blk[:, None] == blk[None, :]
    Ab = np.where(same, A, 0.0)
    pattern = Ab != 0
    assert np.max(np.abs((L @ U - Ab)[pattern])) <= 1e-13 * np.abs(A).max()
    assert np.all(F[~same] == 0)
    assert len(np.unique(blk)) == 3 * 3 * 2   # 19, 17, 11 cells: 3, 3, 2 blocks of 8 positions
    z = np.random.default_rng(13).normal(size=N)
    x = np.linalg.solve(U, np.linalg.solve(L, z))
    assert np.allclose(ilu.apply(z), x, rtol=1e-11, atol=1e-13)


def test_alternating_smoother_step_order():
    """One C-AMS iteration with two post-smoothing steps of the alternating
    smoother: the first step takes the blocks at the origin, the second the
    shifted blocks (composed here step by step)."""
    pb = small_problem(16, 12, 10, (4, 4, 5), sigma=2.0)
    T, P, W, diag, r, LU, piv = _setup(pb, FE)
    A0, A1 = oracle.smoother_for(pb, W, diag, oracle.SMOOTH_BLOCK_ALT)
    d, its, _ = oracle.cams_solve(pb, W, diag, P, FE, LU, piv, (A0, A1), r, n_pre=0, n_post=2,
                                  rtol=1e-30, maxit=1)
    assert its == -1
    d1 = oracle.prolong(pb, P, oracle.lu_solve(LU, piv, oracle.restrict(pb, P, FE, r)))
    r1 = r - oracle.matvec(pb, W, diag, d1)
    e = A0.apply(r1)
    e = e + A1.apply(r1 - oracle.matvec(pb, W, diag, e))
    assert np.allclose(d, d1 + e, rtol=1e-12, atol=1e-14 * np.abs(d).max())
    swapped = d1 + A1.apply(r1)
    swapped = swapped + A0.apply(r1 - oracle.matvec(pb, W, diag, swapped - d1))
    assert not np.allclose(d, swapped, rtol=1e-6)


def test_config1_newton_alternating_smoother_matches_direct_newton():
    """As above with the alternating block smoother (pre- and post-smoothing)."""
    pb = config1()
    T = oracle.transmissibility(pb)
    P = oracle.basis_b4(pb, T)
    p0 = pb.initial_pressure()
    p, rc, st = oracle.newton_step(pb, T, P, p0, p0, lin_rtol=1e-13, newton_tol=1e-12,
                                   smoother=oracle.SMOOTH_BLOCK_ALT)
    assert rc == 0
    ref, _ = helpers.direct_newton(pb, T, p0, p0, tol=1e-12)
    assert np.max(np.abs(p - ref)) <= 1e-10 * np.abs(ref).max()


def test_shift_on_a_single_block_axis_changes_nothing():
    """An axis no longer than a block is one block for any offset: the
    shifted factor equals the unshifted one there (8 x 8 x 8 grid)."""
    pb = small_problem(8, 8, 8, 4, sigma=2.0)
    T = oracle.transmissibility(pb)
    p = np.random.default_rng(14).uniform(0, 1, pb.n)
    W, diag, r, _ = oracle.linear_system(pb, T, p, pb.initial_pressure())
    a = oracle.ILU0(pb, W, diag, block=(8, 8, 8))
    b = oracle.ILU0(pb, W, diag, block=(8, 8, 8), shift=(4, 4, 4))
    for u, v in zip(a.export(), b.export()):
        assert np.array_equal(u, v)


def test_full_dual_blocks_by_brute_force():
    """Full dual blocks = 7x7x7 cells strictly between vertex planes 8 apart
    on every axis; counted by enumerating every cell triple of vertex
    coordinates on a grid with ragged last blocks."""
    pb = small_problem(37, 30, 26, 8, seed=2)
    starts = oracle.full_dual_blocks(pb)
    axes = []
    for n in (pb.nx, pb.ny, pb.nz):
        v = [a * 8 + min(8, n - a * 8) // 2 for a in range((n + 7) // 8)]
        axes.append([v[a] + 1 for a in range(len(v) - 1) if v[a + 1] - v[a] == 8])
    expect = [(x, y, z) for z in axes[2] for y in axes[1] for x in axes[0]]
    assert [tuple(s) for s in starts] == expect and len(expect) > 1


def test_basis_block_ratio_pins():
    """The learned-basis check ||(T Phi)_I|| / ||T_IF Phi_F|| over full dual
    blocks: ~0 for the exact B4 basis (the interior equations hold), exactly
    1 with the interiors zeroed ((T Phi)_I = -T_IF Phi_F), linear in a
    perturbation of the exact basis, and for a perturbation d at one cell c
    with six interior neighbours the squared ratio is proportional to
    (sum_f T_f)^2 + sum_f T_f^2 (the perturbed row and its six neighbours),
    so two cells' ratios compare by their transmissibilities alone."""
    pb = small_problem(24, 24, 16, 8, seed=6, sigma=2.0)
    T = oracle.transmissibility(pb)
    P = oracle.basis_b4(pb, T)
    starts = oracle.full_dual_blocks(pb)
    assert len(starts) == 4
    r_exact = oracle.basis_block_ratios(pb, T, P, starts)
    assert np.all(r_exact <= 1e-12)
    Pz = P.copy().reshape(8, pb.nz, pb.ny, pb.nx)
    for (x0, y0, z0) in starts:
        Pz[:, z0:z0 + 7, y0:y0 + 7, x0:x0 + 7] = 0.0
    r_zero = oracle.basis_block_ratios(pb, T, Pz.reshape(8, -1), starts)
    assert np.allclose(r_zero, 1.0, rtol=1e-13)

    x0, y0, z0 = starts[0]

    def bumped(cells, d):
        Q = P.copy().reshape(8, pb.nz, pb.ny, pb.nx)
        for (i, j, k) in cells:
            Q[3, k, j, i] += d
        return oracle.basis_block_ratios(pb, T, Q.reshape(8, -1), starts[:1])[0]

    def K(i, j, k):
        Tx, Ty, Tz = (T[a].reshape(pb.nz, pb.ny, pb.nx) for a in range(3))
        tf = [Tx[k, j, i - 1], Tx[k, j, i], Ty[k, j - 1, i], Ty[k, j, i], Tz[k - 1, j, i], Tz[k, j, i]]
        return sum(tf) ** 2 + sum(t * t for t in tf)

    a = (x0 + 2, y0 + 3, z0 + 3)
    b = (x0 + 4, y0 + 2, z0 + 4)
    ra, rb = bumped([a], 1e-3), bumped([b], 1e-3)
    assert abs(bumped([a], 2e-3) / ra - 2.0) <= 1e-8
    assert abs((ra / rb) ** 2 - K(*a) / K(*b)) <= 1e-8 * K(*a) / K(*b)


def test_norm_history_incompressible_error_equals_residual():
    """c = 0 (constant density rho0 = 1, dV = 1): F is affine in p and its
    linearisation is exact, so F(p + d) = F(p) + A d = -(r0 - A d) and the
    nonlinear error of every iterate equals the linear residual:
    ||eps(p + d_i)|| = ||r_i|| along the whole history, and one Newton
    iteration suffices."""
    pb = small_problem(16, 12, 8, 4, seed=5, sigma=2.0, c=0.0)
    T = oracle.transmissibility(pb)
    P = oracle.basis_b4(pb, T)
    p0 = pb.initial_pressure()
    p, nu, res, err = oracle.newton_history(pb, T, P, p0, p0, lin_rtol=1e-10, newton_tol=1e-8)
    assert set(nu.tolist()) == {0} and len(res) >= 3
    assert np.allclose(err, res, rtol=1e-9, atol=1e-14 * res[0])
    assert np.all(np.diff(res[:3]) < 0)


def test_norm_history_entries():
    """c > 0: the first entry of each Newton iteration is the Newton error
    ||eps(p^nu)|| and the residual ||r0|| of its system; each linear solve
    stops at its tolerance (relative 1e-1, the paper's adaptive strategy) and
    only there; the step ends with ||eps|| <= 1e-6."""
    pb = small_problem(16, 12, 8, 4, seed=5, sigma=2.0, c=0.1)
    T = oracle.transmissibility(pb)
    P = oracle.basis_b4(pb, T)
    p0 = pb.initial_pressure()
    p, nu, res, err = oracle.newton_history(pb, T, P, p0, p0, lin_rtol=1e-1, newton_tol=1e-6)
    assert oracle.nonlinear_residual(pb, T, p, p0)[1] <= 1e-6
    q = p0.copy()
    for v in range(nu.max() + 1):
        idx = np.nonzero(nu == v)[0]
        W, diag, r0, e = oracle.linear_system(pb, T, q, p0)
        assert abs(err[idx[0]] - e) <= 1e-13 * e and abs(res[idx[0]] - np.linalg.norm(r0)) <= 1e-13 * res[idx[0]]
        assert res[idx[-1]] <= 0.1 * res[idx[0]] and np.all(res[idx[:-1]] > 0.1 * res[idx[0]])
        LU, piv = oracle.lu_factor(oracle.coarse_operator(pb, W, diag, P, pb.restriction))
        d, its, _ = oracle.cams_solve(pb, W, diag, P, pb.restriction, LU, piv, oracle.smoother_for(pb, W, diag),
                                      r0, rtol=1e-1)
        assert its == len(idx) - 1
        q = q + d


def test_absolute_linear_tolerance():
    """lin_atol stops the C-AMS iteration at ||r|| <= atol whatever ||r0||."""
    pb = small_problem(16, 12, 8, 4, seed=5, sigma=2.0, c=0.1)
    T = oracle.transmissibility(pb)
    P = oracle.basis_b4(pb, T)
    p0 = pb.initial_pressure()
    W, diag, r0, _ = oracle.linear_system(pb, T, p0, p0)
    LU, piv = oracle.lu_factor(oracle.coarse_operator(pb, W, diag, P, pb.restriction))
    ilu = oracle.smoother_for(pb, W, diag)
    atol = 1e-6 * np.linalg.norm(r0)
    d, its, hist = oracle.cams_solve(pb, W, diag, P, pb.restriction, LU, piv, ilu, r0, rtol=1e-300, atol=atol)
    assert its > 0
    assert np.linalg.norm(r0 - oracle.matvec(pb, W, diag, d)) <= atol
    assert hist[its - 1] * np.linalg.norm(r0) > atol


def _acc_src(pb, p, pn):
    rho = pb.rho0 * np.exp(pb.c * (p - pb.p0))
    rhon = pb.rho0 * np.exp(pb.c * (pn - pb.p0))
    dV = pb.dx * pb.dy * pb.dz
    src = rho * pb.q * dV if pb.q is not None else 0.0
    return pb.phi * dV * (rho - rhon) / pb.dt, src, pb.phi * pb.c * rhon * dV / pb.dt


def test_face_fluxes_rebuild_the_residual():
    """F_n = accumulation + net outflow of the two-point fluxes - source on
    every non-Dirichlet cell (Eq. (2) cell by cell), with the fluxes
    antisymmetric by construction (one value per face)."""
    pb = small_problem(13, 11, 7, (3, 4, 2), seed=4, sigma=2.0, c=0.1)
    T = oracle.transmissibility(pb)
    rng = np.random.default_rng(3)
    p = rng.uniform(0, 1, pb.n)
    pn = rng.uniform(0, 1, pb.n)
    F_ref, _ = oracle.nonlinear_residual(pb, T, p, pn)
    acc, src, _ = _acc_src(pb, p, pn)
    F = acc + oracle.cell_outflow(pb, oracle.face_flux(pb, T, p)) - src
    free = pb.dirichlet_mask() == 0
    assert np.allclose(F[free], F_ref[free], rtol=1e-12, atol=1e-13 * np.abs(F_ref).max())


@pytest.mark.parametrize("c", [0.0, 0.1])
def test_msfv_sweep_balances_every_coarse_block(c):
    """After MSFE Newton to a loose tolerance, one MSFV stage makes the fluxes
    of the linear system conservative on every primal coarse block: the
    block sums of (accumulation linearised at p + net outflow - source)
    vanish to rounding, where before the sweep they were of the size of the
    Newton error (Sec. 4.2 strategy; MSFV conservation, Sec. 4).  For c = 0
    the linearisation is exact, so the nonlinear block balance also
    vanishes."""
    pb = small_problem(24, 24, 16, 8, seed=9, sigma=2.0, c=c)
    T = oracle.transmissibility(pb)
    P = oracle.basis_b4(pb, T)
    p0 = pb.initial_pressure()
    p, rc, st = oracle.newton_step(pb, T, P, p0, p0, lin_rtol=1e-3, newton_tol=1e-5)
    assert rc == 0
    before = np.abs(oracle.block_balance(pb, T, p, p0)).max()
    p_new, d, flux = oracle.conservative_sweep(pb, T, P, p, p0)
    acc, src, acc_lin = _acc_src(pb, p, p0)
    lin = acc + acc_lin * d + oracle.cell_outflow(pb, flux) - src
    free = pb.dirichlet_mask() == 0
    blk = np.bincount(oracle.primal_block(pb)[free], weights=lin[free], minlength=oracle.num_coarse(pb))
    scale = np.abs(acc).max() + np.abs(flux).max()
    assert before > 1e3 * 1e-14 * scale
    assert np.abs(blk).max() <= 1e-14 * scale * 64
    if c == 0.0:
        assert np.abs(oracle.block_balance(pb, T, p_new, p0)).max() <= 1e-14 * scale * 64


def test_b2_at_uniform_pressure_is_b4():
    """B2 (Eq. (9)) weights the couplings by the face densities of the
    iterate; at a uniform pressure they are T times one constant, and the
    local problems (homogeneous equations with lumped couplings) are
    invariant under that scaling: B2 = B4."""
    pb = small_problem(19, 17, 11, (4, 3, 5), seed=3, sigma=2.0, c=0.2)
    T = oracle.transmissibility(pb)
    p = np.full(pb.n, 0.37)
    C, a = oracle.basis_operator(pb, T, oracle.B2, p=p, pn=p)
    assert a is None
    assert np.abs(oracle.basis_general(pb, C) - oracle.basis_b4(pb, T)).max() <= 1e-14


def test_b3_edge_closed_form_and_no_partition_of_unity():
    """Homogeneous medium (unit transmissibility), B3 (Eq. (10)): along a dual
    edge of 7 cells between vertices 8 apart, (a + 2) Phi_m - Phi_{m-1} -
    Phi_{m+1} = 0 with Phi_0 = 1, Phi_8 = 0, so Phi_m = sinh(th (8 - m)) /
    sinh(8 th) with cosh th = 1 + a / 2 (a = phi c dV / dt).  With the
    accumulation the basis no longer sums to one away from the vertices
    (it does for B2, whose rows sum to zero)."""
    pb = small_problem(16, 16, 16, 8, seed=1, c=0.1, dt=0.1)
    pb.perm = np.ones(pb.n)
    pb.phi = np.full(pb.n, 0.2)
    T = oracle.transmissibility(pb)
    C, a = oracle.basis_operator(pb, T, oracle.B3)
    P = oracle.basis_general(pb, C, a)
    a0 = 0.2 * 0.1 / 0.1
    th = np.arccosh(1.0 + a0 / 2.0)
    m = np.arange(1, 8)
    cells = [pb.cell(4 + k, 4, 4) for k in m]
    assert np.allclose(P[0, cells], np.sinh(th * (8 - m)) / np.sinh(8 * th), rtol=1e-12, atol=1e-15)
    lv = oracle.cell_levels(pb)
    inner = lv < 3
    assert np.all(P.sum(axis=0)[inner] < 1.0 - 1e-6)
    rng = np.random.default_rng(2)
    p = rng.uniform(0, 1, pb.n)
    C2, _ = oracle.basis_operator(pb, T, oracle.B2, p=p, pn=p)
    assert np.allclose(oracle.basis_general(pb, C2).sum(axis=0), 1.0, atol=1e-13)


def test_newton_step_basis_b4_equals_c_newton():
    """The Python Newton loop with a basis type (used for B1-B3) reduces to
    the C Newton step for B4 (same iterates, same count)."""
    pb = small_problem(16, 12, 8, 4, seed=8, sigma=2.0, c=0.1)
    T = oracle.transmissibility(pb)
    p0 = pb.initial_pressure()
    p1, nit, lits = oracle.newton_step_basis(pb, T, p0, p0, oracle.B4, 1e-10, 1e-9)
    p2, rc, st = oracle.newton_step(pb, T, oracle.basis_b4(pb, T), p0, p0, lin_rtol=1e-10, newton_tol=1e-9)
    assert rc == 0 and nit == st["newton_iters"] and lits == st["lin_iters"]
    assert np.array_equal(p1, p2)


@pytest.mark.parametrize("layered", [False, True])
def test_face_dirichlet_series_profile(layered):
    """Pressure fixed on the west (1) and east (0) faces, no flow elsewhere,
    incompressible (c = 0), no wells: steady 1D flow along x.  With the
    half-cell transmissibility 2 k / dx between a cell centre and a boundary
    face, the two-point scheme reproduces the series-resistance profile
    exactly: flux q = 1 / sum_i dx / k_i, and p at cell i = 1 - q (sum_{j<i}
    dx / k_j + dx / (2 k_i)) (homogeneous: 1 - (i + 1/2) / nx)."""
    nx, ny, nz = 12, 3, 2
    pb = small_problem(nx, ny, nz, (4, 3, 2), seed=1, c=0.0, wells="none")
    kx = np.linspace(0.5, 3.0, nx) ** 2 if layered else np.ones(nx)
    pb.perm = np.tile(kx, ny * nz)
    pb.face_bc = {"W": 1.0, "E": 0.0}
    T = oracle.transmissibility(pb)
    p, _ = helpers.direct_newton(pb, T, np.zeros(pb.n), np.zeros(pb.n), tol=1e-13)
    R = 1.0 / kx                        # dx = 1
    q = 1.0 / R.sum()
    ref = 1.0 - q * (np.concatenate([[0.0], np.cumsum(R)[:-1]]) + 0.5 * R)
    assert np.allclose(p.reshape(nz, ny, nx), ref[None, None, :], rtol=0, atol=1e-12)
