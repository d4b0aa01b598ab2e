"""Benchmark of the C-AMS pressure solve on one MI355X.

Workload (one "step"): the 3D 64x64x32 problem with coarsening 8^3, log-
normal permeability (sigma 3), porosity U[0.1,0.3], c = 0.05, corner column
wells: transmissibilities, B4 basis, then 10 backward-Euler time steps of
dt = 0.05, each Newton iteration solving its linear system by C-AMS to a
1e-8 relative residual (Newton to ||eps||_2 <= 1e-8).

Metric: seconds per Newton linear solve = (timed wall time of K steps) /
(number of Newton linear solves in them), inputs resident in HBM.

Prints one JSON line.  --gpus N with N > 1 exits: this build runs on one GPU.
"""

from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def run_workload(solver, pb, torch):
    """One pass of the whole hot path over the workload; returns stats."""
    from paper_1705_05783_amd import _cams as C
    import ctypes
    # new rock => transmissibilities and basis are rebuilt inside the step
    solver.reset_rock()
    pn = solver.new_pressure()
    p = pn.clone()
    solves = 0
    iters = 0
    for _ in range(pb.n_steps):
        st = solver.newton_step(pn, p)
        solves += st["newton_iters"]
        iters += st["lin_iters_total"]
        pn.copy_(p)
    return solves, iters, p


def cpu_baseline(pb):
    """The oracle (single-threaded C) on a bounded sample of the workload:
    one Newton linear solve of the first time step (assembly, coarse
    operator and LU, ILU(0), C-AMS to 1e-8)."""
    import numpy as np
    import oracle
    T = oracle.transmissibility(pb)
    P = oracle.basis_b4(pb, T)
    pn = pb.initial_pressure()
    t0 = time.perf_counter()
    W, diag, r0, _ = oracle.linear_system(pb, T, pn, pn)
    LU, piv = oracle.lu_factor(oracle.coarse_operator(pb, W, diag, P, pb.restriction))
    ilu = oracle.smoother_for(pb, W, diag)
    d, its, _ = oracle.cams_solve(pb, W, diag, P, pb.restriction, LU, piv, ilu, r0)
    dt = time.perf_counter() - t0
    return {"value": dt, "unit": "s per Newton linear solve", "cores": 1, "kind": "oracle",
            "sample": f"one Newton linear solve (first iteration of time step 1) of the 64x64x32 workload, "
                      f"{its} C-AMS iterations to 1e-8; basis excluded; CPU {_cpu_model()}, "
                      f"{len(os.sched_getaffinity(0))} host cores available, oracle is single-threaded"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch
    from workloads import config2
    from paper_1705_05783_amd.solver import Solver

    pb = config2()
    dev = torch.device("cuda:0")
    solver = Solver(pb, device=dev)
    for _ in range(args.warmup):
        run_workload(solver, pb, torch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solves = iters = 0
    for _ in range(args.steps):
        s, i, _ = run_workload(solver, pb, torch)
        solves += s
        iters += i
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1e3 / args.steps
    value = elapsed / max(solves, 1)
    out = {
        "metric": "s per Newton linear solve to 1e-8 rel. residual",
        "value": value,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "64x64x32 lognormal (sigma 3), coarsening 8^3, MSFE, 5 block-ILU(0) "
                               "post-smoothing steps, 10 backward-Euler steps dt=0.05, FP64",
                   "cells": pb.n, "coarse_nodes": solver.Nc,
                   "newton_solves_per_step": solves / args.steps,
                   "cams_iterations_per_solve": iters / max(solves, 1)},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(pb)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
