"""Write the oracle's reference pressures of the 64x64x32 workload.

Calls only `oracle/` (plain FP64 C): the first two backward-Euler steps of
the 64x64x32 workload (lognormal sigma 3, coarsening 8^3, MSFE, alternating
block ILU(0) post-smoothing), each Newton iteration's linear system solved by
C-AMS to a 1e-12 relative residual and Newton run to ||eps||_2 <= 1e-12, so
that the stored pressures carry the 1e-10 relative accuracy the plain FP64
GPU solve is held to.  (1e-12 rather than tighter: the first linear system
of step 2 stalls at about 2e-13 relative residual, the rounding level of
its FP64 residual.)  The oracle needs about 100 s per step on one core,
too long for a parity test, hence the stored result.

Output: config2_plain_steps.npz (pressure after step 1 and after step 2)
and config2_plain_steps.json (settings, oracle statistics and a SHA-256 of
the generated inputs, so that a test can tell when the workload generator
has changed and the file is stale).

Run from the repository root:  python tests/golden/make_reference_pressures.py
"""

from __future__ import annotations

import hashlib
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

LIN_RTOL = 1e-12
NEWTON_TOL = 1e-12
STEPS = 2


def input_digest(pb) -> str:
    h = hashlib.sha256()
    for a in (pb.perm, pb.phi, pb.dirichlet_mask(), pb.initial_pressure()):
        h.update(np.ascontiguousarray(a).tobytes())
    h.update(repr((pb.nx, pb.ny, pb.nz, pb.rx, pb.ry, pb.rz, pb.c, pb.dt, pb.restriction, pb.n_post,
                   pb.smoother)).encode())
    return h.hexdigest()


def main():
    import oracle
    from workloads import config2
    pb = config2()
    T = oracle.transmissibility(pb)
    P = oracle.basis_b4(pb, T)
    pn = pb.initial_pressure()
    out, stats = {}, []
    for step in range(1, STEPS + 1):
        p, rc, st = oracle.newton_step(pb, T, P, pn, pn, lin_rtol=LIN_RTOL, newton_tol=NEWTON_TOL)
        if rc != 0:
            raise RuntimeError(f"oracle Newton failed at step {step}: {rc}")
        out[f"step{step}"] = p
        stats.append(st)
        print(f"step {step}: {st}", flush=True)
        pn = p
    np.savez(os.path.join(HERE, "config2_plain_steps.npz"), **out)
    meta = {"workload": "64x64x32 lognormal sigma 3, coarsening 8^3, MSFE, alternating block ILU(0), "
                        "10 steps of dt 0.05 (first two stored)",
            "lin_rtol": LIN_RTOL, "newton_tol": NEWTON_TOL, "steps": STEPS, "oracle_stats": stats,
            "inputs_sha256": input_digest(pb)}
    with open(os.path.join(HERE, "config2_plain_steps.json"), "w") as f:
        json.dump(meta, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
