"""Basis types B1-B3 (Sec. 3, Eqs. (8)-(10)) and their adaptive updates.

The local problems of every type run through the same GPU kernel (face
couplings plus an optional diagonal); the basis of each type is compared
with the oracle's at a given iterate, and whole time steps with the oracle's
Newton loop that rebuilds B1/B2 at every iteration.  The adaptive update
(regions re-solved when their coefficients changed by more than basis_tol)
must reach the same pressure, since C-AMS is iterated to the tolerance with
whatever basis it holds, and must re-solve fewer regions than the full
rebuild.
"""

import numpy as np
import pytest

import oracle
from tests.gpu_util import log, rel_err, require_gpu, solver_for, to_np
from workloads import small_problem

pytestmark = pytest.mark.gpu

KINDS = {"B1": oracle.B1, "B2": oracle.B2, "B3": oracle.B3}


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.mark.parametrize("kind", ["B1", "B2", "B3"])
@pytest.mark.parametrize("shape,r", [((24, 24, 16), 8), ((19, 17, 11), (4, 3, 5)), ((13, 11, 1), (3, 4, 1))])
def test_basis_types_match_oracle(torch, kind, shape, r):
    pb = small_problem(*shape, r, sigma=2.0, seed=71, c=0.2, dt=0.05)
    pb.basis_type = KINDS[kind]
    s = solver_for(pb)
    rng = np.random.default_rng(5)
    p = pb.initial_pressure()
    free = pb.dirichlet_mask() == 0
    p[free] = rng.uniform(0, 1, free.sum())
    pn = pb.initial_pressure()
    s.assemble(torch.as_tensor(p, device="cuda"), torch.as_tensor(pn, device="cuda"))
    s.build_basis()
    P = to_np(s.export(4)).reshape(8, -1)
    T = oracle.transmissibility(pb)
    P_ref = oracle.basis_general(pb, *oracle.basis_operator(pb, T, KINDS[kind], p=p, pn=pn))
    err = np.abs(P - P_ref).max()
    log(pb.name, kind, "max |P - P_ref|", err, "column sums", P_ref.sum(axis=0).min(), P_ref.sum(axis=0).max())
    assert err <= 1e-12
    s.close()


@pytest.mark.parametrize("kind", ["B1", "B2", "B3"])
def test_newton_with_basis_type(torch, kind):
    """One time step with linear solves to 1e-12 and Newton to 1e-11: B1/B2
    rebuilt at every Newton iteration (basis_tol 0), B3 once; pressure
    against the oracle's Newton with the same rule to 1e-10."""
    pb = small_problem(24, 24, 16, 8, sigma=2.0, seed=72, c=0.2, dt=0.05).with_options(
        lin_rtol=1e-12, newton_tol=1e-11)
    pb.basis_type = KINDS[kind]
    s = solver_for(pb)
    p0 = pb.initial_pressure()
    pn_t = torch.as_tensor(p0, device="cuda")
    p_t = pn_t.clone()
    st = s.newton_step(pn_t, p_t)
    T = oracle.transmissibility(pb)
    p_ref, nit, lits = oracle.newton_step_basis(pb, T, p0, p0, KINDS[kind], 1e-12, 1e-11)
    err = rel_err(to_np(p_t), p_ref)
    log(kind, "gpu newton", st["newton_iters"], "cams", st["lin_iters_total"], "updates", st["basis_updates"],
        "regions", st["basis_regions_rebuilt"], "| oracle newton", nit, "cams", lits, "| err", err)
    assert err <= 1e-10 and abs(st["newton_iters"] - nit) <= 1
    if kind in ("B1", "B2"):
        assert st["basis_updates"] == st["newton_iters"] - 1
    s.close()


def test_adaptive_basis_update(torch):
    """B1 with the update threshold at 0 (every region, every iteration), at
    1e30 (never after the first build) and in between: all reach the
    oracle's pressure (1e-9 relative at linear 1e-12 / Newton 1e-11); the
    intermediate threshold re-solves more regions than the frozen basis and
    fewer than the full rebuild."""
    base = small_problem(32, 32, 24, 8, sigma=2.5, seed=73, c=0.2, dt=0.05).with_options(
        lin_rtol=1e-12, newton_tol=1e-11, basis_type=oracle.B1)
    T = oracle.transmissibility(base)
    p0 = base.initial_pressure()
    p_ref, nit, _ = oracle.newton_step_basis(base, T, p0, p0, oracle.B1, 1e-12, 1e-11)
    rebuilt = {}
    for tol in (0.0, 0.02, 1e30):
        pb = base.with_options(basis_tol=tol)
        s = solver_for(pb)
        pn_t = torch.as_tensor(p0, device="cuda")
        p_t = pn_t.clone()
        st = s.newton_step(pn_t, p_t)
        err = rel_err(to_np(p_t), p_ref)
        rebuilt[tol] = st["basis_regions_rebuilt"]
        log("basis_tol", tol, "newton", st["newton_iters"], "cams", st["lin_iters_total"], "regions re-solved",
            st["basis_regions_rebuilt"], "updates", st["basis_updates"], "err", err)
        assert err <= 1e-9
        s.close()
    assert rebuilt[1e30] < rebuilt[0.02] < rebuilt[0.0]


@pytest.mark.parametrize("wells", ["none", "corners"])
def test_face_dirichlet_newton(torch, wells):
    """Dirichlet west / east faces (the paper's default boundary conditions),
    with or without the corner well columns: one time step at linear 1e-12 /
    Newton 1e-11 against the oracle's Newton, 1e-10."""
    pb = small_problem(24, 24, 16, 8, sigma=2.0, seed=74, c=0.1, dt=0.05, wells=wells).with_options(
        lin_rtol=1e-12, newton_tol=1e-11, face_bc={"W": 1.0, "E": 0.0})
    s = solver_for(pb)
    p0 = pb.initial_pressure()
    pn_t = torch.as_tensor(p0, device="cuda")
    p_t = pn_t.clone()
    st = s.newton_step(pn_t, p_t)
    T = oracle.transmissibility(pb)
    p_ref, rc, ost = oracle.newton_step(pb, T, oracle.basis_b4(pb, T), p0, p0, lin_rtol=1e-12, newton_tol=1e-11)
    err = rel_err(to_np(p_t), p_ref)
    log("face bc", wells, "gpu", st["newton_iters"], st["lin_iters_total"], "oracle", ost, "err", err)
    assert rc == 0 and err <= 1e-10
    _, e = oracle.nonlinear_residual(pb, T, to_np(p_t), p0)
    assert e <= 1e-11
    s.close()
