"""Benchmark of the C-AMS pressure solve on one MI355X.

Workload (one "step"): the 3D 64x64x32 problem with coarsening 8^3, log-
normal permeability (sigma 3), porosity U[0.1,0.3], c = 0.05, corner column
wells: transmissibilities, B4 basis, then 10 backward-Euler time steps of
dt = 0.05, each Newton iteration solving its linear system by C-AMS to a
1e-8 relative residual (Newton to ||eps||_2 <= 1e-8).

Metric: seconds per Newton linear solve = (timed wall time of K steps) /
(number of Newton linear solves in them), inputs resident in HBM.  The
headline value is the mixed-precision solve (FP32 smoother, basis storage
and prolongation; FP64 residual, update and coarse solve); the plain FP64
solve of the same workload is timed beside it.

Prints one JSON line.  --gpus N with N > 1 exits: the solve runs on one GPU.
"""

from __future__ import annotations

import argparse
import json

import numpy as np
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


PEAK_HBM_GBS = 8000.0   # MI355X HBM3E
LEARNED_FALLBACK_TOL = 10.0   # a network block is re-solved when its basis residual exceeds 10x its boundary flux


def timed_run(pb, steps, warmup, torch):
    """Warm up, then time `steps` whole-workload passes; the smoothing-step
    kernel is timed by the library with HIP events on its stream."""
    from paper_1705_05783_amd.solver import Solver
    solver = Solver(pb, device=torch.device("cuda:0"))
    for _ in range(warmup):
        run_workload(solver, pb, torch)
    torch.cuda.synchronize()
    solver.profile()
    t0 = time.perf_counter()
    solves = iters = 0
    for _ in range(steps):
        s, i, _ = run_workload(solver, pb, torch)
        solves += s
        iters += i
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = solver.profile_read()
    return {"elapsed": elapsed, "solves": solves, "iters": iters, "prof": prof, "Nc": solver.Nc}


def batch_run(steps, warmup, torch, sequential=True):
    """256 uneven instances (nx, ny ~ U{32..96}, nz ~ U{16..48}, ratios
    U{4..8}, sigma U[1,4], c U[0.01,0.2]; seed 3), mixed precision, one
    Newton iteration each (basis, assembly, coarse operator, C-AMS to 1e-8,
    update) per batched step; the batched iterations are one launch per
    kernel over all instances.  The same instances solved one after another
    by the single-problem path are timed once for comparison."""
    from paper_1705_05783_amd.batch import Batch
    from workloads.configs import batch_problems
    pbs = batch_problems()
    sizes = [pb.n for pb in pbs]
    flat_pn = torch.as_tensor(np.concatenate([pb.initial_pressure() for pb in pbs]), device="cuda")
    flat_p = flat_pn.clone()
    offs = np.concatenate([[0], np.cumsum(sizes)])
    pn = [flat_pn[offs[i]:offs[i + 1]] for i in range(len(pbs))]
    p = [flat_p[offs[i]:offs[i + 1]] for i in range(len(pbs))]
    b = Batch.from_problems(pbs)

    def step():
        for sv in b.solvers:
            sv.invalidate_basis()
        flat_p.copy_(flat_pn)
        status, stats = b.newton_iteration(pn, p)
        if any(s != 0 for s in status):
            raise RuntimeError(f"batched solve failed: {sorted(set(status))}")
        return stats

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        stats = step()
    torch.cuda.synchronize()
    elapsed = (time.perf_counter() - t0) / steps
    its = np.array([st["lin_iters_last"] for st in stats])
    out = {"workload": "256 uneven 3D instances (16k-411k cells), mixed precision, one Newton iteration each",
           "instances": len(pbs), "cells": int(sum(sizes)), "s_per_batch_step": elapsed,
           "instances_per_s": len(pbs) / elapsed, "cells_per_s": sum(sizes) / elapsed,
           "cams_iterations": {"min": int(its.min()), "mean": float(its.mean()), "max": int(its.max())},
           "setup_ms": stats[0]["t_coarse_ms"], "iterate_ms": stats[0]["t_iterate_ms"], "tuning": b.tuning()}
    if sequential:
        # the same instances, one at a time through the single-problem path
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i, sv in enumerate(b.solvers):
            sv.invalidate_basis()
            p[i].copy_(pn[i])
            sv.newton_step(pn[i], p[i], check=False)
        torch.cuda.synchronize()
        seq = time.perf_counter() - t0
        out["sequential_single_path_s"] = seq
        out["speedup_vs_sequential"] = seq / elapsed
    b.close()
    return out


def large_run(torch):
    """The 256x256x128 channelised workload (8.4M cells, 16384 coarse nodes,
    block-tridiagonal coarse factorisation), BF16 basis and prolongation,
    FP32 smoother, FP64 residual and coarse solve: one pass of its 5 time
    steps, smoother kernel timed live."""
    from paper_1705_05783_amd.solver import Solver
    from workloads.configs import config4
    pb = config4()
    solver = Solver(pb, device=torch.device("cuda:0"))
    solver.profile()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solves, iters, _ = run_workload(solver, pb, torch)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    out = {"workload": "256x256x128 channelised (k 1 / 1e-4, 30% channels), coarsening 8^3, 16384 coarse nodes, "
                       "BF16 basis, 5 time steps dt=0.05 to 1e-8",
           "cells": pb.n, "coarse_nodes": solver.Nc, "s_per_solve": elapsed / max(solves, 1),
           "ms_per_pass": elapsed * 1e3, "newton_solves": solves,
           "cams_iterations_per_solve": iters / max(solves, 1),
           "roofline_smoother": roofline(solver.profile_read(), "256x256x128 channelised BF16")}
    solver.close()
    return out


def learned_run(torch):
    """The 128^3 evaluation workload (sigma 3, correlation 8, c = 0.1, one
    time step): time to solution per Newton linear solve for plain FP64
    C-AMS, mixed precision, and mixed precision with the trained network for
    the full dual-block interiors (local-solve fallback for blocks whose
    basis residual exceeds LEARNED_FALLBACK_TOL times their boundary flux).
    The basis is rebuilt in every pass, so its cost is in the per-solve
    time."""
    import torch as _t
    from paper_1705_05783_amd import _cams as C
    from paper_1705_05783_amd.solver import Solver
    from paper_1705_05783_amd.train_basis import load_weights
    from workloads.configs import FP64, MIXED_FP32, config5_eval
    params = load_weights()
    out = {"workload": "128^3 lognormal (sigma 3, corr. 8), coarsening 8^3, c=0.1, one time step, Newton and "
                       "linear solves to 1e-8"}
    for label, prec, learned in (("plain_fp64", FP64, False), ("mixed", MIXED_FP32, False),
                                 ("learned_mixed", MIXED_FP32, True)):
        pb = config5_eval(precision=prec)
        solver = Solver(pb, device=_t.device("cuda:0"))
        if learned:
            solver.set_learned(params, fallback_tol=LEARNED_FALLBACK_TOL)
        run_workload(solver, pb, torch)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solves, iters, _ = run_workload(solver, pb, torch)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        r = {"s_per_solve": elapsed / max(solves, 1), "newton_solves": solves,
             "cams_iterations_per_solve": iters / max(solves, 1)}
        if learned:
            r.update(solver.basis_stats())
        out[label] = r
        solver.close()
    out["speedup_learned_mixed_vs_plain"] = out["plain_fp64"]["s_per_solve"] / out["learned_mixed"]["s_per_solve"]
    out["speedup_mixed_vs_plain"] = out["plain_fp64"]["s_per_solve"] / out["mixed"]["s_per_solve"]
    # basis error of the network against the exact local solves (FP64 storage)
    pb = config5_eval(precision=FP64)
    solver = Solver(pb, device=_t.device("cuda:0"))
    solver.build_basis()
    P_exact = solver.export(C.CAMS_ARR_P)
    solver.set_learned(params, fallback_tol=1e30)
    solver.build_basis()
    P_net = solver.export(C.CAMS_ARR_P)
    out["basis_rel_l2_error_no_fallback"] = float((P_net - P_exact).norm() / P_exact.norm())
    solver.close()
    return out


def measured_traffic(workload):
    """HBM bytes per launch of the smoother kernel from the committed memory
    counter record (FETCH_SIZE + WRITE_SIZE, scaled by a device copy), or
    None when the kernel source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_k_bilu_step.json")
    try:
        rec = json.load(open(path))
        src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    except (OSError, ValueError, KeyError):
        return None
    if hashlib.sha256(src).hexdigest() != rec.get("source_sha256"):
        return None
    w = rec["workloads"].get(workload)
    return None if w is None else w["traffic_bytes_per_launch"]


def roofline(prof, workload=None):
    if prof["launches"] == 0 or prof["total_ms"] <= 0:
        return None
    per_launch_bytes = prof["bytes"] / prof["launches"]
    avg_s = prof["total_ms"] * 1e-3 / prof["launches"]
    achieved = per_launch_bytes / avg_s / 1e9
    return {"kernel": "k_bilu_step (block-ILU(0) Richardson step)", "bound": "hbm",
            "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
            "traffic": measured_traffic(workload) if workload else None, "avg_launch_us": avg_s * 1e6,
            "bytes_per_launch": per_launch_bytes, "launches": prof["launches"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["mixed", "plain", "both", "batch", "large", "learned", "copy"],
                    default="both",
                    help="mixed/plain/both: the headline workload; batch/large/learned: that workload alone "
                         "(one JSON object, for profiling); copy: a 256 MiB device copy, the reference kernel "
                         "for scaling memory counters")
    ap.add_argument("--no-batch", action="store_true", help="skip the 256-instance batched solve")
    ap.add_argument("--no-extra", action="store_true", help="skip the large and learned-basis workloads")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the solve runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch
    from workloads import config2
    from workloads.configs import FP64, MIXED_FP32

    if args.only == "copy":
        a = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copies": 3}), flush=True)
        return
    if args.only in ("batch", "large", "learned"):
        fn = {"batch": lambda: batch_run(args.steps, args.warmup, torch, sequential=False),
              "large": lambda: large_run(torch), "learned": lambda: learned_run(torch)}[args.only]
        print(json.dumps({args.only: fn()}), flush=True)
        return

    runs = {}
    if args.only in ("mixed", "both"):
        runs["mixed"] = timed_run(config2(precision=MIXED_FP32), args.steps, args.warmup, torch)
    if args.only in ("plain", "both"):
        runs["plain"] = timed_run(config2(precision=FP64), args.steps, args.warmup, torch)
    head = runs.get("mixed") or runs["plain"]
    pb = config2()

    def summary(r):
        return {"s_per_solve": r["elapsed"] / max(r["solves"], 1),
                "ms_per_step": r["elapsed"] * 1e3 / args.steps,
                "newton_solves_per_step": r["solves"] / args.steps,
                "cams_iterations_per_solve": r["iters"] / max(r["solves"], 1),
                "roofline_smoother": roofline(r["prof"])}

    out = {
        "metric": "s per Newton linear solve to 1e-8 rel. residual",
        "value": head["elapsed"] / max(head["solves"], 1),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["elapsed"] * 1e3 / args.steps,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if "mixed" in runs else "f64",
        "data": "synthetic",
        "config": {"workload": "64x64x32 lognormal (sigma 3, corr. 8x8x2), coarsening 8^3 (256 coarse nodes), "
                               "MSFE, 5 block-ILU(0) post-smoothing steps (block grid shifted by half a block on every other "
                               "step), 10 backward-Euler steps dt=0.05, "
                               "Newton and linear solves to 1e-8; value = mixed precision (FP32 smoother, "
                               "basis and prolongation, FP64 residual/update/coarse solve)" if "mixed" in runs
                               else "64x64x32 workload, plain FP64",
                   "cells": pb.n, "coarse_nodes": head["Nc"],
                   "newton_solves_per_step": head["solves"] / args.steps,
                   "cams_iterations_per_solve": head["iters"] / max(head["solves"], 1)},
        "roofline": roofline(head["prof"], "64x64x32 mixed" if "mixed" in runs else None),
    }
    for k, r in runs.items():
        out[k] = summary(r)
    if "mixed" in runs and "plain" in runs:
        out["speedup_mixed_vs_plain_per_solve"] = (runs["plain"]["elapsed"] / runs["plain"]["solves"]) / \
            (runs["mixed"]["elapsed"] / runs["mixed"]["solves"])
    if not args.no_batch:
        out["batch"] = batch_run(args.steps, args.warmup, torch)
    if not args.no_extra:
        out["large"] = large_run(torch)
        out["learned"] = learned_run(torch)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(pb)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
