"""Benchmark of the C-AMS pressure solve on one MI355X.

Headline workload: the 128^3 learned-basis evaluation field (ln k lognormal,
sigma 3, correlation length 8 cells, seed 5; coarsening 8^3 = 4096 coarse
nodes; porosity 0.2, c = 0.1, dt = 0.1, corner column wells; MSFE; 5
alternating block-ILU(0) post-smoothing steps; Newton and linear solves to
1e-8).  One "step" = one pass of the whole hot path over it: new rock
(transmissibilities), basis, then one backward-Euler time step whose Newton
iterations each assemble, build the coarse operator and its inverse, and
solve the linear system by C-AMS.  Three variants run the same pass:

  plain_fp64      FP64 throughout, basis by exact local solves;
  mixed           FP32 smoother, basis storage and prolongation, FP64
                  residual, update and coarse solve (iterative refinement);
  learned_mixed   mixed, with the trained network for the interiors of the
                  full dual blocks (exact re-solve of blocks whose local
                  equation ratio exceeds the calibrated fallback tolerance).

Metric: seconds per Newton linear solve to a 1e-8 relative residual =
median pass wall time / Newton linear solves per pass (time to solution per
solve: the basis is rebuilt in every pass and counted), inputs resident in
HBM.  value = learned_mixed; plain_fp64 and mixed beside it, with the
iterations-only time per solve (hipEvent around the C-AMS iterations).
The roofline object is the smoother step, the kernel with the largest total
time in the learned_mixed pass, timed live with HIP events on the library's
stream.  The other workloads (64x64x32, the 256x256x128 channelised field,
the 256-instance batch) follow as extra keys with the same --steps/--warmup.

Prints one JSON line.  --gpus N with N > 1 exits: the solve runs on one GPU.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0   # MI355X HBM3E


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def run_pass(solver, pb):
    """One pass of the hot path: rock (and so basis) reset, then every time
    step of the workload.  Returns per-pass totals from the library's stats."""
    solver.reset_rock()
    pn = solver.new_pressure()
    p = pn.clone()
    out = {"solves": 0, "iters": 0, "t_iterate_ms": 0.0, "t_basis_ms": 0.0, "t_coarse_ms": 0.0,
           "t_assemble_ms": 0.0, "fallback_blocks": 0, "coarse_factorizations": 0, "basis_rebuilds": 0}
    for _ in range(pb.n_steps):
        st = solver.newton_step(pn, p)
        out["solves"] += st["newton_iters"]
        out["iters"] += st["lin_iters_total"]
        for k in ("t_iterate_ms", "t_basis_ms", "t_coarse_ms", "t_assemble_ms"):
            out[k] += st[k]
        out["fallback_blocks"] = max(out["fallback_blocks"], st["fallback_blocks"])
        out["coarse_factorizations"] += st["coarse_factorizations"]
        out["basis_rebuilds"] += st["basis_rebuilds"]
        pn.copy_(p)
    return out


def timed_passes(solver, pb, steps, warmup, torch):
    """`warmup` untimed passes, then `steps` passes each timed on the wall
    clock (synchronised on both sides); the smoother step is timed by the
    library with HIP events on its stream during the timed passes."""
    for _ in range(warmup):
        run_pass(solver, pb)
    torch.cuda.synchronize()
    solver.profile()
    walls, stats = [], []
    t_all = time.perf_counter()
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = run_pass(solver, pb)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        stats.append(st)
    total = time.perf_counter() - t_all
    prof = solver.profile_read()
    solves = stats[0]["solves"]
    assert all(s["solves"] == solves for s in stats), "passes differ in their Newton iterations"
    med = float(np.median(walls))
    return {"s_per_solve": med / max(solves, 1),
            "ms_per_pass_median": med * 1e3, "ms_per_pass_min": min(walls) * 1e3,
            "ms_per_pass_max": max(walls) * 1e3, "passes": steps, "total_s": total,
            "newton_solves_per_pass": solves,
            "cams_iterations_per_solve": stats[0]["iters"] / max(solves, 1),
            "iterate_ms_per_solve_median": float(np.median([s["t_iterate_ms"] / max(s["solves"], 1)
                                                            for s in stats])),
            "basis_ms_median": float(np.median([s["t_basis_ms"] for s in stats])),
            "coarse_ms_per_solve_median": float(np.median([s["t_coarse_ms"] / max(s["solves"], 1)
                                                          for s in stats])),
            "fallback_blocks": stats[0]["fallback_blocks"],
            "basis_rebuilds": sum(s["basis_rebuilds"] for s in stats),
            "coarse_factorizations_per_pass": stats[0]["coarse_factorizations"], "prof": prof}


def measured_traffic(workload):
    """HBM bytes per launch of the smoother step from the committed memory
    counter record (FETCH_SIZE + WRITE_SIZE, scaled by a device copy), or
    None when the kernel source has changed since the counters were taken."""
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


# The smoothing-step kernel each precision and grid size launches: one
# workgroup per 8^3 block with register sweeps while all blocks are resident
# at once (64x64x32), else the LDS sweeps (FP32: four blocks along x per
# workgroup, in one round of resident workgroups at 128^3 and in several
# at 256x256x128; FP64: one block per workgroup).
SMOOTHER_KERNEL = {
    ("resident", "f32"): "k_bilu_step<float, float, 512, 1>",
    ("resident", "f64"): "k_bilu_step<double, double, 512, 1>",
    ("many", "f32"): "k_bilu_step_row<float, float, 4, 512>",
    ("rounds", "f32"): "k_bilu_step_rows<float, float, 4, 512>",
    ("many", "f64"): "k_bilu_step<double, double, 256, 0>",
}


def roofline(prof, workload=None, kernel=None):
    if prof["launches"] == 0 or prof["total_ms"] <= 0:
        return None
    per_launch_bytes = prof["bytes"] / prof["launches"]
    avg_s = prof["total_ms"] * 1e-3 / prof["launches"]
    achieved = per_launch_bytes / avg_s / 1e9
    return {"kernel": f"{kernel} (block-ILU(0) Richardson step)", "bound": "hbm",
            "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
            "traffic": measured_traffic(workload) if workload else None, "avg_launch_us": avg_s * 1e6,
            "bytes_per_launch": per_launch_bytes, "launches": prof["launches"]}


def headline(steps, warmup, torch):
    """The 128^3 workload: plain FP64, mixed and learned+mixed."""
    from paper_1705_05783_amd.solver import Solver
    from paper_1705_05783_amd.train_basis import load_fallback_tol, load_weights
    from workloads.configs import FP64, MIXED_FP32, config5_eval
    params = load_weights()
    tol = load_fallback_tol()
    out = {}
    for label, prec, learned in (("plain_fp64", FP64, False), ("mixed", MIXED_FP32, False),
                                 ("learned_mixed", MIXED_FP32, True)):
        pb = config5_eval(precision=prec)
        solver = Solver(pb)
        guard = 0
        if learned:
            # global check: twice the exact basis' iterations per solve (mixed run)
            guard = int(np.ceil(out["mixed"]["cams_iterations_per_solve"]))
            solver.set_learned(params, fallback_tol=tol, guard_iters=guard)
        r = timed_passes(solver, pb, steps, warmup, torch)
        r["roofline_smoother"] = roofline(r.pop("prof"), f"128^3 {label}",
                                          SMOOTHER_KERNEL["many", "f64" if prec == FP64 else "f32"])
        if learned:
            r["fallback_tol"] = tol
            r["guard_iters"] = guard
            r["full_dual_blocks"] = solver.num_full_blocks()
        r["coarse_nodes"] = solver.Nc
        out[label] = r
        solver.close()
    pl, mx, lm = out["plain_fp64"], out["mixed"], out["learned_mixed"]
    out["speedup_learned_mixed_vs_plain"] = pl["s_per_solve"] / lm["s_per_solve"]
    out["speedup_mixed_vs_plain"] = pl["s_per_solve"] / mx["s_per_solve"]
    out["speedup_learned_mixed_vs_mixed"] = mx["s_per_solve"] / lm["s_per_solve"]
    out["speedup_learned_mixed_vs_plain_iterations_only"] = (pl["iterate_ms_per_solve_median"] /
                                                             lm["iterate_ms_per_solve_median"])
    return out


def adaptive_run(steps, warmup, torch):
    """The paper's linear/nonlinear stopping strategies (Sec. 4.1.1) on the
    headline workload in its learned+mixed form, both to ||eps||_2 < 1e-6:
    each Newton linear system solved to 1e-8 relative residual, against the
    adaptive strategy that updates the system once the residual has dropped
    by one order (linear 1e-1).  Time to solution per pass (one time step)."""
    from paper_1705_05783_amd.solver import Solver
    from paper_1705_05783_amd.train_basis import load_fallback_tol, load_weights
    from workloads.configs import MIXED_FP32, config5_eval
    params = load_weights()
    out = {"workload": "128^3 learned+mixed, one time step per pass, Newton to ||eps||_2 < 1e-6"}
    for label, lin in (("linear_1e-8", 1e-8), ("adaptive_1e-1", 1e-1)):
        pb = config5_eval(precision=MIXED_FP32).with_options(lin_rtol=lin, newton_tol=1e-6)
        solver = Solver(pb)
        solver.set_learned(params, fallback_tol=load_fallback_tol())
        r = timed_passes(solver, pb, steps, warmup, torch)
        r.pop("prof")
        r["s_per_time_step"] = r["ms_per_pass_median"] * 1e-3
        out[label] = r
        solver.close()
    out["speedup_adaptive"] = out["linear_1e-8"]["s_per_time_step"] / out["adaptive_1e-1"]["s_per_time_step"]
    return out


def coarse_reuse_run(steps, warmup, torch):
    """Adaptive coarse factorisation (coarse_tol 0.05: the inverse is kept
    while R A P_hat stays within 5 % of the factorised operator) against
    factorising at every Newton iteration, on the 128^3 learned+mixed
    workload and on the 256x256x128 channelised one."""
    from paper_1705_05783_amd.solver import Solver
    from paper_1705_05783_amd.train_basis import load_fallback_tol, load_weights
    from workloads.configs import MIXED_FP32, config4, config5_eval
    out = {"coarse_tol": 0.05}
    params = load_weights()
    for name, make in (("128^3_learned_mixed", lambda: config5_eval(precision=MIXED_FP32)),
                       ("256x256x128_channelised", config4)):
        pb = make().with_options(coarse_tol=0.05)
        solver = Solver(pb)
        if name.startswith("128"):
            solver.set_learned(params, fallback_tol=load_fallback_tol())
        r = timed_passes(solver, pb, steps, warmup, torch)
        r.pop("prof")
        out[name] = r
        solver.close()
    return out


def small_run(steps, warmup, torch):
    """The 64x64x32 workload (10 time steps of dt 0.05 per pass), mixed and
    plain FP64."""
    from paper_1705_05783_amd.solver import Solver
    from workloads import config2
    from workloads.configs import FP64, MIXED_FP32
    out = {"workload": "64x64x32 lognormal (sigma 3, corr. 8x8x2), coarsening 8^3 (256 coarse nodes), MSFE, "
                       "10 backward-Euler steps dt=0.05 per pass, Newton and linear solves to 1e-8"}
    for label, prec in (("mixed", MIXED_FP32), ("plain_fp64", FP64)):
        pb = config2(precision=prec)
        solver = Solver(pb)
        r = timed_passes(solver, pb, steps, warmup, torch)
        r["roofline_smoother"] = roofline(r.pop("prof"), "64x64x32 mixed" if label == "mixed" else None,
                                          SMOOTHER_KERNEL["resident", "f32" if label == "mixed" else "f64"])
        out[label] = r
        solver.close()
    out["speedup_mixed_vs_plain"] = out["plain_fp64"]["s_per_solve"] / out["mixed"]["s_per_solve"]
    return out


def smoothers_run(steps, warmup, torch):
    """The library's four ILU(0) smoothers (Table "cams" step 6) on the
    64x64x32 workload in FP64 (10 time steps per pass): block-Jacobi on 8^3
    blocks, the same alternating with the half-block-shifted grid,
    red-black, and the paper's global ILU(0) in natural order (a wavefront
    over 16x16x8 bricks, one launch per brick diagonal).  C-AMS iterations
    and seconds per Newton solve."""
    from paper_1705_05783_amd.solver import Solver
    from workloads import config2
    from workloads.configs import FP64, SMOOTH_BLOCK, SMOOTH_BLOCK_ALT, SMOOTH_NATURAL, SMOOTH_REDBLACK
    out = {"workload": "64x64x32 lognormal (sigma 3, corr. 8x8x2), coarsening 8^3 (256 coarse nodes), MSFE, "
                       "FP64, 10 backward-Euler steps dt=0.05 per pass, Newton and linear solves to 1e-8"}
    for label, sm in (("block", SMOOTH_BLOCK), ("block_alt", SMOOTH_BLOCK_ALT), ("red_black", SMOOTH_REDBLACK),
                      ("natural", SMOOTH_NATURAL)):
        pb = config2(precision=FP64).with_options(smoother=sm)
        solver = Solver(pb)
        r = timed_passes(solver, pb, steps, warmup, torch)
        r.pop("prof")
        out[label] = {k: r[k] for k in ("s_per_solve", "cams_iterations_per_solve", "iterate_ms_per_solve_median",
                                        "ms_per_pass_median", "newton_solves_per_pass")}
        out[label]["ms_per_cams_iteration"] = r["iterate_ms_per_solve_median"] / r["cams_iterations_per_solve"]
        solver.close()
    return out


def large_run(steps, warmup, torch):
    """The 256x256x128 channelised workload (8.4M cells, 16384 coarse nodes,
    block-tridiagonal coarse factorisation), BF16 basis and prolongation,
    FP32 smoother, FP64 residual and coarse solve; one pass = its 5 time
    steps."""
    from paper_1705_05783_amd.solver import Solver
    from workloads.configs import config4
    pb = config4()
    solver = Solver(pb)
    r = timed_passes(solver, pb, steps, warmup, torch)
    r["roofline_smoother"] = roofline(r.pop("prof"), "256x256x128 channelised BF16", SMOOTHER_KERNEL["rounds", "f32"])
    r.update({"workload": "256x256x128 channelised (k 1 / 1e-4, 30% channels), coarsening 8^3, 16384 coarse "
                          "nodes, BF16 basis, 5 time steps dt=0.05 per pass, to 1e-8",
              "cells": pb.n, "coarse_nodes": solver.Nc})
    solver.close()
    return r


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
    walls = []
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = step()
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
    med = float(np.median(walls))
    its = np.array([st["lin_iters_last"] for st in stats])
    out = {"workload": "256 uneven 3D instances (16k-411k cells), mixed precision, one Newton iteration each",
           "instances": len(pbs), "cells": int(sum(sizes)), "s_per_batch_step_median": med,
           "instances_per_s": len(pbs) / med, "cells_per_s": sum(sizes) / med, "passes": steps,
           "cams_iterations": {"min": int(its.min()), "mean": float(its.mean()), "max": int(its.max())},
           "setup_ms": stats[0]["t_coarse_ms"], "iterate_ms": stats[0]["t_iterate_ms"], "tuning": b.tuning()}
    # the batched FP32 smoothing step of the chosen form, as the tuner timed it
    # (one launch over every block of every instance; 32 B per cell)
    forms = [(128, 1), (256, 1), (512, 1), (512, 4)]
    t = out["tuning"]
    ms = t["ms_per_smooth_step"][forms.index((t["smoother_threads"], t["smoother_blocks"]))]
    nbytes = 32.0 * sum(sizes)
    gbs = nbytes / (ms * 1e-3) / 1e9
    out["roofline_batched_smoother"] = {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                        "frac": gbs / PEAK_HBM_GBS, "ms_per_step": ms,
                                        "bytes_per_step": nbytes,
                                        "form": f"{t['smoother_threads']} threads, {t['smoother_blocks']} block(s)"}
    if sequential:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i, sv in enumerate(b.solvers):
            sv.invalidate_basis()
            p[i].copy_(pn[i])
            sv.newton_step(pn[i], p[i], check=False)
        torch.cuda.synchronize()
        seq = time.perf_counter() - t0
        out["sequential_single_path_s"] = seq
        out["speedup_vs_sequential"] = seq / med
    b.close()
    return out


def cpu_baseline(gpu_plain):
    """The oracle (plain FP64 C-AMS, the same algorithm as plain_fp64) on the
    128^3 workload, in its timing build (-O3 -march=native -fopenmp, built
    here for this host), on a bounded sample of one pass: transmissibilities,
    the whole B4 basis, then the first Newton iteration's assembly, coarse
    operator R A P, coarse LU, ILU(0) factors and 3 C-AMS iterations.  Per
    Newton linear solve = basis / solves per pass + assembly + coarse
    operator + LU + ILU(0) setup + (C-AMS iterations per solve of the GPU
    plain_fp64 pass, which the oracle's count matches within one) x time per
    iteration.  Two legs: all host cores, and one thread (there the LU is
    timed on the leading 2048 x 2048 block of the coarse operator and scaled
    by 8 = (4096/2048)^3)."""
    import oracle
    from workloads.configs import FP64, config5_eval
    pb = config5_eval(precision=FP64)
    oracle.build_timing()
    cores = min(16, len(os.sched_getaffinity(0)))   # the host share of one GPU
    solves = gpu_plain["newton_solves_per_pass"]
    its = gpu_plain["cams_iterations_per_solve"]
    legs = {}
    for threads in (cores, 1) if cores > 1 else (1,):
        with oracle.timing_build(threads):
            t = {}
            t0 = time.perf_counter()
            T = oracle.transmissibility(pb)
            P = oracle.basis_b4(pb, T)
            t["basis"] = time.perf_counter() - t0
            pn = pb.initial_pressure()
            t0 = time.perf_counter()
            W, diag, r0, _ = oracle.linear_system(pb, T, pn, pn)
            t["assemble"] = time.perf_counter() - t0
            t0 = time.perf_counter()
            Ac = oracle.coarse_operator(pb, W, diag, P, pb.restriction)
            t["coarse_operator"] = time.perf_counter() - t0
            t0 = time.perf_counter()
            if threads == 1 and cores > 1:
                oracle.lu_factor(Ac[:2048, :2048])
                t["coarse_lu"] = 8.0 * (time.perf_counter() - t0)
                LU, piv = legs[cores]["_lu"]
            else:
                LU, piv = oracle.lu_factor(Ac)
                t["coarse_lu"] = time.perf_counter() - t0
            t0 = time.perf_counter()
            ilu = oracle.smoother_for(pb, W, diag)
            t["ilu_setup"] = time.perf_counter() - t0
            t0 = time.perf_counter()
            oracle.cams_solve(pb, W, diag, P, pb.restriction, LU, piv, ilu, r0, maxit=3)
            t["per_iteration"] = (time.perf_counter() - t0) / 3
            per_solve = (t["basis"] / max(solves, 1) + t["assemble"] + t["coarse_operator"] + t["coarse_lu"] +
                         t["ilu_setup"] + its * t["per_iteration"])
            legs[threads] = {"s_per_solve": per_solve, "threads": threads, "parts_s": t, "_lu": (LU, piv)}
    for leg in legs.values():
        leg.pop("_lu")
    best = legs[cores]
    return {"value": best["s_per_solve"], "unit": "s per Newton linear solve", "cores": cores, "kind": "oracle",
            "sample": f"128^3 plain FP64 (the headline workload): B4 basis + first Newton iteration's assembly, "
                      f"R A P, coarse LU (4096 nodes), ILU(0) setup and 3 C-AMS iterations, scaled to "
                      f"{its:.1f} iterations per solve and {solves} solves per pass; oracle timing build "
                      f"-O3 -march=native -fopenmp on {cores} threads; CPU {_cpu_model()}",
            "single_thread": {"value": legs[1]["s_per_solve"], "parts_s": legs[1]["parts_s"],
                              "note": "coarse LU timed on the leading 2048 x 2048 block, x8" if cores > 1
                              else "coarse LU timed in full"},
            "all_cores": {"value": best["s_per_solve"], "threads": cores, "parts_s": best["parts_s"]}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=7, help="timed passes per workload (median reported)")
    ap.add_argument("--warmup", type=int, default=2, help="untimed passes per workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["headline", "adaptive", "coarse", "small", "large", "batch", "smoothers",
                                       "copy", "all"],
                    default="all",
                    help="headline/small/large/batch: that workload alone (one JSON object, for profiling); "
                         "smoothers: the four ILU(0) smoothers on the 64x64x32 workload (not part of 'all'); "
                         "copy: a 256 MiB device copy, the reference kernel for scaling memory counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the solve runs on one GPU; --gpus must be 1", "n_gpus": args.gpus}),
              flush=True)
        sys.exit(2)
    import torch

    if args.only == "copy":
        a = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copies": 3}), flush=True)
        return
    steps, warmup = max(1, args.steps), max(0, args.warmup)
    if args.only in ("adaptive", "coarse", "small", "large", "batch", "smoothers"):
        fn = {"adaptive": adaptive_run, "coarse": coarse_reuse_run, "small": small_run, "large": large_run,
              "batch": lambda s, w, t: batch_run(s, w, t, False), "smoothers": smoothers_run}
        print(json.dumps({args.only: fn[args.only](steps, warmup, torch)}), flush=True)
        return

    t_start = time.perf_counter()

    def progress(leg):   # one line on stderr per finished leg; stdout keeps the single JSON line
        print(f"bench: {leg} done at {time.perf_counter() - t_start:.1f} s", file=sys.stderr, flush=True)

    head = headline(steps, warmup, torch)
    progress("headline (128^3 plain, mixed, learned+mixed)")
    lm = head["learned_mixed"]
    from workloads.configs import config5_eval
    pb = config5_eval()
    out = {
        "metric": "s per Newton linear solve to 1e-8 rel. residual, learned+mixed vs plain; HBM GB/s",
        "value": lm["s_per_solve"],
        "unit": "s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": lm["ms_per_pass_median"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "128^3 lognormal (sigma 3, corr. 8, seed 5), coarsening 8^3 (4096 coarse nodes), "
                               "c=0.1, dt=0.1, one time step per pass, MSFE, 5 alternating block-ILU(0) "
                               "post-smoothing steps, Newton and linear solves to 1e-8; value = learned+mixed "
                               "(trained network for the full dual-block interiors with local-solve fallback, "
                               "FP32 smoother/basis/prolongation, FP64 residual/update/coarse solve), time to "
                               "solution per Newton linear solve incl. the basis",
                   "cells": pb.n, "coarse_nodes": lm["coarse_nodes"],
                   "newton_solves_per_step": lm["newton_solves_per_pass"],
                   "cams_iterations_per_solve": lm["cams_iterations_per_solve"]},
        "roofline": lm["roofline_smoother"],
        "learned_mixed": lm,
        "mixed": head["mixed"],
        "plain_fp64": head["plain_fp64"],
    }
    for k in ("speedup_learned_mixed_vs_plain", "speedup_mixed_vs_plain", "speedup_learned_mixed_vs_mixed",
              "speedup_learned_mixed_vs_plain_iterations_only"):
        out[k] = head[k]
    if args.only == "all":
        for key, fn in (("adaptive_newton", adaptive_run), ("adaptive_coarse", coarse_reuse_run),
                        ("small", small_run), ("large", large_run), ("batch", batch_run)):
            out[key] = fn(steps, warmup, torch)
            progress(key)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(head["plain_fp64"])
        progress("cpu_baseline")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
