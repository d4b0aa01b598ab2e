"""Small cases through every C entry point of the oracle, for the sanitizer
test (tests/test_sanitizers.py).  The oracle library named on the command
line (built with AddressSanitizer and UndefinedBehaviorSanitizer, no
recovery) replaces the normal build; then each case runs once.  A sanitizer
report ends the process with an error; exit status 0 means every case ran
clean.  Not a pytest module: the test runs it in a child process with the
sanitizer runtime preloaded.
"""

import ctypes
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import oracle  # noqa: E402
from workloads import config1, small_problem  # noqa: E402
from workloads.configs import (FE, FV, SMOOTH_BLOCK, SMOOTH_BLOCK_ALT, SMOOTH_NATURAL,  # noqa: E402
                               SMOOTH_REDBLACK)

SMOOTHERS = (SMOOTH_BLOCK, SMOOTH_BLOCK_ALT, SMOOTH_REDBLACK, SMOOTH_NATURAL)


def factors(ilu):
    return ilu if isinstance(ilu, tuple) else (ilu,)


def run():
    rng = np.random.default_rng(0)
    # the 2D workload (MSFV, 5 + 5 smoothing steps) under every smoother
    pb = config1()
    T = oracle.transmissibility(pb)
    P = oracle.basis_b4(pb, T)
    pn = pb.initial_pressure()
    for sm in SMOOTHERS:
        _, rc, _ = oracle.newton_step(pb, T, P, pn, pn, smoother=sm)
        assert rc == 0, ("2D Newton", sm, rc)
    print("2D Newton, four smoothers", flush=True)

    # a ragged 3D grid with mixed coarsening ratios, both restrictions
    pb = small_problem(13, 11, 7, (4, 3, 5), sigma=2.0)
    T = oracle.transmissibility(pb)
    P = oracle.basis_b4(pb, T)
    pn = pb.initial_pressure()
    p = pn.copy()
    free = pb.dirichlet_mask() == 0
    p[free] = rng.uniform(0, 1, free.sum())
    oracle.vertex_coords(pb.nx, pb.rx)
    oracle.cell_levels(pb)
    oracle.slot_nodes(pb)
    oracle.primal_block(pb)
    oracle.nonlinear_residual(pb, T, p, pn)
    W, diag, r, _ = oracle.linear_system(pb, T, p, pn)
    oracle.matvec(pb, W, diag, r)
    for R in (FE, FV):
        Ac = oracle.coarse_operator(pb, W, diag, P, R)
        LU, piv = oracle.lu_factor(Ac)
        oracle.prolong(pb, P, oracle.lu_solve(LU, piv, oracle.restrict(pb, P, R, r)))
        for sm in SMOOTHERS:
            ilu = oracle.smoother_for(pb, W, diag, sm)
            for f in factors(ilu):
                f.apply(r)
                f.export()
            _, its, _ = oracle.cams_solve(pb, W, diag, P, R, LU, piv, ilu, r, rtol=1e-10, maxit=400)
            assert its >= 0, ("3D C-AMS", R, sm)
    print("3D operators, restrictions, smoothers, C-AMS", flush=True)

    # Newton with histories, the conservative sweep and fluxes, basis types
    p1, rc, _ = oracle.newton_step(pb, T, P, pn, pn)
    assert rc == 0
    oracle.newton_history(pb, T, P, pn, pn, 1e-1, 1e-6)
    p2, _, F = oracle.conservative_sweep(pb, T, P, p1, pn)
    oracle.cell_outflow(pb, F)
    oracle.face_flux(pb, T, p2)
    oracle.block_balance(pb, T, p2, pn)
    for kind in (1, 2, 3):
        oracle.basis_operator(pb, T, kind, p=p1, pn=pn)
        oracle.newton_step_basis(pb, T, pn, pn, kind, 1e-8, 1e-8)
    print("histories, conservative sweep, fluxes, basis types B1-B3", flush=True)

    # Dirichlet boundary faces, and a 1D chain (exact natural-order ILU)
    pb = small_problem(12, 10, 6, 3, sigma=1.5).with_options(face_bc={"W": 1.0, "E": 0.0})
    T = oracle.transmissibility(pb)
    P = oracle.basis_b4(pb, T)
    pn = pb.initial_pressure()
    _, rc, _ = oracle.newton_step(pb, T, P, pn, pn)
    assert rc == 0
    from workloads import Problem
    n = 17
    chain = Problem("chain", n, 1, 1, 3, 1, 1, np.exp(rng.normal(0, 1, n)), np.full(n, 0.2), [(0, 1.0)],
                    c=0.1, dt=0.5)
    T = oracle.transmissibility(chain)
    W, diag, _, _ = oracle.linear_system(chain, T, rng.uniform(0, 1, n), chain.initial_pressure())
    oracle.smoother_for(chain, W, diag, SMOOTH_NATURAL).apply(rng.normal(size=n))
    print("boundary faces, 1D chain", flush=True)


if __name__ == "__main__":
    oracle._lib = oracle._configure(ctypes.CDLL(sys.argv[1]))
    run()
    print("oracle cases done", flush=True)
