"""MSFE to convergence, then one MSFV sweep with two-point flux
reconstruction (cams_conservative_sweep; Sec. 4.2 and the conservation
property of MSFV stated in Sec. 4).

Parity: from the same pressure, the GPU's MSFV correction and fluxes
against the oracle's conservative_sweep.  Property at any size: after MSFE
Newton convergence, the sweep's fluxes balance the linearised accumulation
and the sources on every primal coarse block to rounding (the oracle sums
them per block), where before the sweep the blocks are out of balance by
about the Newton tolerance.
"""

import numpy as np
import pytest

import oracle
from tests.gpu_util import log, rel_err, require_gpu, solver_for, to_np
from workloads import small_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _linearised_block_balance(pb, T, p, pn, d, flux):
    """Per primal block: accumulation at p + its linearisation times d +
    net outflow of the fluxes - sources, over the non-Dirichlet cells; and
    the magnitude scale of those terms."""
    rho = pb.rho0 * np.exp(pb.c * (p - pb.p0))
    rhon = pb.rho0 * np.exp(pb.c * (pn - pb.p0))
    dV = pb.dx * pb.dy * pb.dz
    acc = pb.phi * dV * (rho - rhon) / pb.dt + pb.phi * pb.c * rhon * dV / pb.dt * d
    src = rho * pb.q * dV if pb.q is not None else 0.0
    lin = acc + oracle.cell_outflow(pb, flux) - src
    free = pb.dirichlet_mask() == 0
    blk = np.bincount(oracle.primal_block(pb)[free], weights=lin[free], minlength=oracle.num_coarse(pb))
    scale = np.abs(pb.phi * dV * (rho + rhon) / pb.dt).max() + np.abs(flux).max()
    return blk, scale


@pytest.mark.parametrize("shape,r,precision", [((24, 24, 16), 8, 0), ((19, 17, 11), (4, 3, 5), 0),
                                               ((24, 24, 16), 8, 1), ((20, 20, 1), 4, 0)])
def test_sweep_matches_oracle(torch, shape, r, precision):
    """From a pressure one loose Newton iteration away from the initial one
    (residual far above rounding), the GPU sweep's update and fluxes match
    the oracle's: the coarse MSFV inverse (LU with partial pivoting) against
    the oracle's LU solve, to 1e-9 relative; the fluxes to 1e-9 of their
    largest value."""
    pb = small_problem(*shape, r, sigma=2.0, seed=61, c=0.1).with_options(lin_rtol=1e-2, newton_maxit=1)
    pb.precision = precision
    s = solver_for(pb)
    p0 = pb.initial_pressure()
    pn_t = torch.as_tensor(p0, device="cuda")
    p_t = pn_t.clone()
    s.newton_step(pn_t, p_t, check=False)
    p1 = to_np(p_t)
    flux = to_np(s.conservative_sweep(pn_t, p_t))
    d_gpu = to_np(p_t) - p1
    T = oracle.transmissibility(pb)
    P = to_np(s.export(4)).reshape(8, -1)    # the basis in use (rounded in mixed precision)
    p_ref, d_ref, flux_ref = oracle.conservative_sweep(pb, T, P, p1, p0)
    log(pb.name, "precision", precision, "d err", rel_err(d_gpu, d_ref), "flux err", rel_err(flux, flux_ref))
    assert rel_err(d_gpu, d_ref) <= 1e-9
    assert rel_err(flux, flux_ref) <= 1e-9
    s.close()


@pytest.mark.parametrize("workload", ["64x64x32", "128^3_learned_mixed"])
def test_sweep_conserves_after_msfe_convergence(torch, workload):
    """The paper's recommended finish at full size: MSFE Newton to 1e-8
    (64x64x32 plain FP64; the 128^3 learned+mixed workload with 4096 coarse
    nodes), then one MSFV sweep: every primal coarse block balances to
    rounding (<= 1e-12 of the term scale), from an imbalance before the
    sweep well above that."""
    from workloads import config2
    from workloads.configs import config5_eval
    if workload == "64x64x32":
        pb = config2()
        s = solver_for(pb)
    else:
        from paper_1705_05783_amd.train_basis import load_fallback_tol, load_weights
        pb = config5_eval()
        s = solver_for(pb)
        s.set_learned(load_weights(), fallback_tol=load_fallback_tol())
    pn_t = s.new_pressure()
    p_t = pn_t.clone()
    st = s.newton_step(pn_t, p_t)
    p = to_np(p_t)
    pn = to_np(pn_t)
    T = oracle.transmissibility(pb)
    before = np.abs(oracle.block_balance(pb, T, p, pn)).max()
    flux = to_np(s.conservative_sweep(pn_t, p_t))
    d = to_np(p_t) - p
    blk, scale = _linearised_block_balance(pb, T, p, pn, d, flux)
    log(workload, "newton", st["newton_iters"], "imbalance before", before, "after", np.abs(blk).max(),
        "scale", scale)
    assert np.abs(blk).max() <= 1e-12 * scale
    assert before > 10 * np.abs(blk).max()
    # the fluxes are those of the two-point scheme at the new pressure with the densities of p
    assert rel_err(flux, oracle.face_flux(pb, T, to_np(p_t), p_rho=p)) <= 1e-12
    s.close()


def test_sweep_rejects_block_tridiagonal_grids(torch):
    from paper_1705_05783_amd import _cams as C
    pb = small_problem(96, 96, 40, 4, sigma=2.0, seed=31, c=0.1)
    s = solver_for(pb)
    assert C.cams_coarse_planes(s.ctx) > 0
    p = s.new_pressure()
    with pytest.raises(C.CamsError) as e:
        s.conservative_sweep(p.clone(), p)
    assert e.value.status == C.CAMS_E_ARG
    s.close()
