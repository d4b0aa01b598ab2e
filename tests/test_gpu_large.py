"""Large coarse grids and the full-size channelised workload.

Block-tridiagonal coarse factorisation (MSFE, > 4096 coarse nodes): the
oracle's coarse operator is checked to be block tridiagonal over coarse
z-planes (exact zeros elsewhere), the GPU coarse operator matches it to
1e-12, and the GPU coarse solve matches a LAPACK solve of the oracle's
operator (relative error <= 1e-8, residual <= 1e-10).  At the full
256x256x128 size (8.4M cells, 16384 coarse nodes, BF16 basis) one Newton
iteration is checked through a property that holds at any size: the
oracle recomputes r0 - A delta on its own FP64 matrix and finds
||r|| <= lin_rtol ||r0|| (1% slack for the different summation order).
"""

import numpy as np
import pytest

import oracle
from tests.gpu_util import log, rel_err, require_gpu, solver_for, to_np
from workloads import small_problem
from workloads.configs import config4

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


# (grid, seed): 10 coarse z-planes (elimination chains of 4 and 5 planes
# around the twist plane), 3 (one plane each side), 4 (one above, two below)
# and 5 planes of 1024 nodes (the block GEMVs' 16-byte row loads)
@pytest.mark.parametrize("shape,seed", [((96, 96, 40), 31), ((160, 160, 12), 33), ((144, 144, 16), 34),
                                        ((128, 128, 20), 37)])
def test_blocktri_coarse_operator_and_solve(torch, shape, seed):
    from paper_1705_05783_amd import _cams as C
    pb = small_problem(*shape, 4, sigma=2.0, seed=seed, c=0.1)
    s = solver_for(pb)
    nbx, Z = shape[0] // 4, shape[2] // 4
    m = nbx * (shape[1] // 4)
    assert C.cams_coarse_planes(s.ctx) == Z and s.Nc == Z * m
    p0 = torch.as_tensor(pb.initial_pressure(), device="cuda")
    s.assemble(p0, p0.clone())
    s.build_basis()
    s.coarse_op()
    T = oracle.transmissibility(pb)
    P = oracle.basis_b4(pb, T)
    W, diag, r0, _ = oracle.linear_system(pb, T, pb.initial_pressure(), pb.initial_pressure())
    Ac = oracle.coarse_operator(pb, W, diag, P, pb.restriction)
    plane = np.arange(s.Nc) // m
    far = np.abs(plane[:, None] - plane[None, :]) > 1
    assert np.count_nonzero(Ac[far]) == 0   # block tridiagonal over coarse z-planes
    # and within the coupling of adjacent planes, 9-point: the plane products use it
    node = np.arange(s.Nc) % m
    ax, by = node % nbx, node // nbx
    spread = (np.abs(ax[:, None] - ax[None, :]) > 1) | (np.abs(by[:, None] - by[None, :]) > 1)
    assert np.count_nonzero(Ac[~far & spread]) == 0
    Ac_gpu = to_np(s.export(C.CAMS_ARR_AC)).reshape(s.Nc, s.Nc)
    assert rel_err(Ac_gpu, Ac) <= 1e-12
    rng = np.random.default_rng(seed)
    rc = rng.normal(size=s.Nc)
    xc = to_np(s.coarse_solve(torch.as_tensor(rc, device="cuda")))
    ref = np.linalg.solve(Ac, rc)
    err = rel_err(xc, ref)
    res = np.linalg.norm(Ac @ xc - rc) / np.linalg.norm(rc)
    log("blocktri coarse solve: rel err", err, "residual", res)
    assert err <= 1e-8 and res <= 1e-10
    s.close()


def test_dense_coarse_solve_at_4096_nodes(torch):
    """4096 coarse nodes, the largest dense MSFE inverse (Gauss-Jordan sweeps
    whose update launches take the lean GEMM tile) and the dense coarse GEMV
    with 16-byte row loads: the GPU coarse solve against a LAPACK solve of
    the oracle's operator."""
    from paper_1705_05783_amd import _cams as C
    pb = small_problem(64, 64, 64, 4, sigma=2.0, seed=36, c=0.1)
    s = solver_for(pb)
    assert C.cams_coarse_planes(s.ctx) == 0 and s.Nc == 4096
    p0 = torch.as_tensor(pb.initial_pressure(), device="cuda")
    s.assemble(p0, p0.clone())
    s.build_basis()
    s.coarse_op()
    rng = np.random.default_rng(36)
    rc = rng.normal(size=s.Nc)
    xc = to_np(s.coarse_solve(torch.as_tensor(rc, device="cuda")))
    s.close()
    T = oracle.transmissibility(pb)
    P = oracle.basis_b4(pb, T)
    W, diag, r0, _ = oracle.linear_system(pb, T, pb.initial_pressure(), pb.initial_pressure())
    Ac = oracle.coarse_operator(pb, W, diag, P, pb.restriction)
    err = rel_err(xc, np.linalg.solve(Ac, rc))
    res = np.linalg.norm(Ac @ xc - rc) / np.linalg.norm(rc)
    log("dense 4096 coarse solve: rel err", err, "residual", res)
    assert err <= 1e-8 and res <= 1e-10


def test_blocktri_on_a_caller_stream(torch):
    """The second elimination chain forks from and joins back to the stream
    the context was created on; here a stream of the caller's own (not the
    default one), with the solve right after the factorisation on it."""
    pb = small_problem(144, 144, 16, 4, sigma=2.0, seed=35, c=0.1)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        s = solver_for(pb, stream=st)
        p0 = torch.as_tensor(pb.initial_pressure(), device="cuda")
        s.assemble(p0, p0.clone())
        s.build_basis()
        s.coarse_op()
        rng = np.random.default_rng(35)
        rc = rng.normal(size=s.Nc)
        xc = to_np(s.coarse_solve(torch.as_tensor(rc, device="cuda")))
        s.close()
    T = oracle.transmissibility(pb)
    P = oracle.basis_b4(pb, T)
    W, diag, r0, _ = oracle.linear_system(pb, T, pb.initial_pressure(), pb.initial_pressure())
    Ac = oracle.coarse_operator(pb, W, diag, P, pb.restriction)
    err = rel_err(xc, np.linalg.solve(Ac, rc))
    log("blocktri on a caller stream: rel err", err)
    assert err <= 1e-8


def test_blocktri_linear_solve_meets_tolerance(torch):
    pb = small_problem(96, 96, 40, 4, sigma=2.0, seed=32, c=0.1).with_options(lin_rtol=1e-10, newton_maxit=1)
    s = solver_for(pb)
    p0 = pb.initial_pressure()
    p = torch.as_tensor(p0, device="cuda")
    st = s.newton_step(p.clone(), p, check=False)
    log("blocktri newton iteration", st)
    T = oracle.transmissibility(pb)
    W, diag, r0, _ = oracle.linear_system(pb, T, p0, p0)
    r = r0 - oracle.matvec(pb, W, diag, to_np(p) - p0)
    rel = np.linalg.norm(r) / np.linalg.norm(r0)
    assert st["newton_iters"] == 1 and rel <= 1e-10 * 1.01, rel
    s.close()


def test_config4_full_size_one_newton_iteration(torch):
    """256x256x128 channelised field, BF16 basis and prolongation, FP32
    smoother, FP64 residual and block-tridiagonal coarse solve."""
    from paper_1705_05783_amd import _cams as C
    pb = config4().with_options(newton_maxit=1)
    s = solver_for(pb)
    assert C.cams_coarse_planes(s.ctx) == 16
    p0 = pb.initial_pressure()
    p = torch.as_tensor(p0, device="cuda")
    st = s.newton_step(p.clone(), p, check=False)
    log("config4 one Newton iteration", st)
    T = oracle.transmissibility(pb)
    W, diag, r0, e0 = oracle.linear_system(pb, T, p0, p0)
    r = r0 - oracle.matvec(pb, W, diag, to_np(p) - p0)
    rel = np.linalg.norm(r) / np.linalg.norm(r0)
    assert st["newton_iters"] == 1 and rel <= pb.lin_rtol * 1.01, rel
    _, e1 = oracle.nonlinear_residual(pb, T, to_np(p), p0)
    log("eps before", e0, "after", e1)
    assert e1 < 0.1 * e0
    s.close()
