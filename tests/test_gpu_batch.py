"""Batched solve (cams_batch_*) against the oracle and the single-problem path.

Every instance of a batch must compute what one Newton iteration of its own
problem computes: the oracle's Newton update (one iteration, linear solves
to 1e-12 on both sides: relative error of the update <= 1e-9), and the
single-problem path's result (same kernels and the same order of operations
per instance: relative difference <= 1e-12, equal iteration counts).  At
the full 256-instance size every instance's residual is recomputed by the
oracle (||r0 - A delta|| <= lin_rtol ||r0|| up to rounding) and sampled
instances are compared with the single-problem path.
"""

import numpy as np
import pytest

import oracle
from tests.gpu_util import linear_residual_check, log, rel_err, require_gpu, to_np
from workloads import small_problem
from workloads.configs import FE, FP64, FV, MIXED_BF16, MIXED_FP32, SMOOTH_BLOCK, SMOOTH_BLOCK_ALT, batch_problems

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _instances(precision, n_pre=0, rtol=1e-12, alt=False):
    """Uneven shapes, ratios and restrictions, one instance at rest; with
    `alt` every other instance takes the alternating block smoother."""
    specs = [
        ((16, 12, 8), 4, FE, dict(sigma=2.0, seed=3, c=0.1)),
        ((19, 17, 11), (4, 3, 5), FE, dict(sigma=2.5, seed=4, c=0.05)),
        ((24, 24, 16), 8, FE, dict(sigma=3.0, seed=5, c=0.2)),
        ((10, 9, 12), (2, 3, 2), FV, dict(sigma=1.5, seed=6, c=0.01)),
        ((8, 8, 8), 8, FE, dict(sigma=1.0, seed=7, c=0.1)),
        ((33, 21, 17), (5, 4, 6), FV, dict(sigma=2.0, seed=8, c=0.1)),
        ((20, 20, 1), 4, FE, dict(sigma=2.0, seed=9, c=0.1)),
        ((16, 12, 8), 4, FE, dict(sigma=2.0, seed=10, c=0.1, wells="none")),   # at rest: r0 = 0
    ]
    out = []
    for q, (shape, r, restr, kw) in enumerate(specs):
        pb = small_problem(*shape, r, restriction=restr, n_pre=n_pre, **kw)
        pb = pb.with_options(precision=precision, lin_rtol=rtol, newton_maxit=1,
                             smoother=SMOOTH_BLOCK_ALT if alt and q % 2 == 0 else SMOOTH_BLOCK)
        out.append(pb)
    return out


def _start(pb):
    p = pb.initial_pressure()
    if not pb.wells:
        p = np.full(pb.n, 0.3)
    return p


def _run_batch(torch, pbs):
    from paper_1705_05783_amd.batch import Batch
    b = Batch.from_problems(pbs)
    pn = [torch.as_tensor(_start(pb), device="cuda") for pb in pbs]
    p = [t.clone() for t in pn]
    status, stats = b.newton_iteration(pn, p)
    return b, status, stats, [to_np(t) for t in p]


def _oracle_update(pb, lin_rtol):
    T = oracle.transmissibility(pb)
    P = oracle.basis_b4(pb, T)
    p0 = _start(pb)
    p, rc, st = oracle.newton_step(pb, T, P, p0, p0, lin_rtol=lin_rtol, newton_maxit=1)
    return p - p0, st


@pytest.mark.parametrize("precision,alt", [(FP64, False), (MIXED_FP32, False), (MIXED_BF16, False),
                                           (FP64, True), (MIXED_FP32, True)])
def test_batch_matches_oracle(torch, precision, alt):
    pbs = _instances(precision, alt=alt)
    b, status, stats, p = _run_batch(torch, pbs)
    log("batch", precision, status, [s["lin_iters_last"] for s in stats], b.tuning())
    for pb, s, st, pg in zip(pbs, status, stats, p):
        assert s == 0, (pb.name, s)
        d_gpu = pg - _start(pb)
        if not pb.wells:
            assert st["lin_iters_last"] == 0 and np.max(np.abs(d_gpu)) == 0.0
            continue
        d_ref, ost = _oracle_update(pb, 1e-12)
        err = rel_err(d_gpu, d_ref)
        log(pb.name, "iters", st["lin_iters_last"], "oracle", ost["lin_iters"], "err", err)
        assert err <= 1e-9, pb.name
        assert st["relres_last"] <= 1e-12
    b.close()


@pytest.mark.parametrize("precision,n_pre,alt", [(FP64, 0, False), (FP64, 2, False), (MIXED_FP32, 1, False),
                                                 (MIXED_BF16, 0, False), (FP64, 3, True), (MIXED_FP32, 0, True)])
def test_batch_matches_single_path(torch, precision, n_pre, alt):
    from paper_1705_05783_amd.solver import Solver
    pbs = _instances(precision, n_pre=n_pre, rtol=1e-8, alt=alt)
    b, status, stats, p = _run_batch(torch, pbs)
    for pb, s, st, pg in zip(pbs, status, stats, p):
        assert s == 0, (pb.name, s)
        sv = Solver(pb)
        pn = torch.as_tensor(_start(pb), device="cuda")
        ps = pn.clone()
        single = sv.newton_step(pn, ps, check=False)
        first = single["lin_iters_total"] if single["newton_iters"] else 0
        diff = rel_err(pg, to_np(ps))
        log(pb.name, "batch iters", st["lin_iters_last"], "single", first, "diff", diff)
        assert st["lin_iters_last"] == first, pb.name
        assert diff <= 1e-12, pb.name
        sv.close()
    b.close()


@pytest.mark.parametrize("form", [(128, 1), (256, 1), (512, 1), (512, 4)])
def test_batch_smoother_forms_match_single_path(torch, form):
    """Every smoother form the tuner can pick (threads, blocks per
    workgroup), fixed by cams_batch_set_smoother, gives the single path's
    iteration counts and pressures (1e-12) on the mixed-precision batch with
    the alternating smoother (the four-block form stages the shifted grid's
    wrapped blocks too)."""
    from paper_1705_05783_amd.batch import Batch
    from paper_1705_05783_amd.solver import Solver
    pbs = _instances(MIXED_FP32, rtol=1e-8, alt=True)
    b = Batch.from_problems(pbs)
    b.set_smoother(*form)
    pn = [torch.as_tensor(_start(pb), device="cuda") for pb in pbs]
    p = [t.clone() for t in pn]
    status, stats = b.newton_iteration(pn, p)
    t = b.tuning()
    assert (t["smoother_threads"], t["smoother_blocks"]) == form
    for pb, s, st, pg in zip(pbs, status, stats, p):
        assert s == 0, (pb.name, s)
        sv = Solver(pb)
        q0 = torch.as_tensor(_start(pb), device="cuda")
        q = q0.clone()
        single = sv.newton_step(q0, q, check=False)
        first = single["lin_iters_total"] if single["newton_iters"] else 0
        diff = rel_err(to_np(pg), to_np(q))
        log(pb.name, form, "batch iters", st["lin_iters_last"], "single", first, "diff", diff)
        assert st["lin_iters_last"] == first, pb.name
        assert diff <= 1e-12, pb.name
        sv.close()
    b.close()


def test_batch_smoother_form_rejects_invalid_pairs(torch):
    from paper_1705_05783_amd import _cams as C
    from paper_1705_05783_amd.batch import Batch
    b = Batch.from_problems(_instances(FP64, rtol=1e-8))
    for bad in ((512, 4), (64, 1), (512, 2)):   # (512, 4) is FP32 only
        with pytest.raises(C.CamsError) as e:
            b.set_smoother(*bad)
        assert e.value.status == C.CAMS_E_ARG
    b.set_smoother(0, 0)
    b.close()


def test_batch_second_call_replays_the_tuned_graph(torch):
    """The second call runs the chosen graph only; it must reproduce the first
    call's result bit for bit from the same starting state."""
    from paper_1705_05783_amd.batch import Batch
    pbs = _instances(MIXED_FP32, rtol=1e-8)
    b = Batch.from_problems(pbs)
    pn = [torch.as_tensor(_start(pb), device="cuda") for pb in pbs]
    runs = []
    for rep in range(2):
        p = [t.clone() for t in pn]
        status, stats = b.newton_iteration(pn, p)
        assert all(s == 0 for s in status)
        runs.append(([to_np(t) for t in p], [s["lin_iters_last"] for s in stats]))
    t = b.tuning()
    log("tuning", t)
    assert t["iters_per_graph"] in (2, 4, 8)
    forms = [(128, 1), (256, 1), (512, 1), (512, 4)]   # (threads, blocks) per workgroup
    assert (t["smoother_threads"], t["smoother_blocks"]) in forms
    # the tuner keeps the fastest smoother form it measured (the four-block
    # form only in FP32: this batch is mixed, so all four are measured)
    ms = t["ms_per_smooth_step"]
    assert all(m > 0 for m in ms)
    assert ms[forms.index((t["smoother_threads"], t["smoother_blocks"]))] == min(ms)
    assert runs[0][1] == runs[1][1]
    for a, c in zip(runs[0][0], runs[1][0]):
        assert np.array_equal(a, c)
    b.close()


def test_tuning_cache_reuses_the_choice(torch):
    """The process-wide tuning cache.  After it is cleared, a batch times its
    candidates (from_cache 0) and stores the outcome; a second batch with
    the same key (new contexts; same precision, smoothing counts and size
    buckets) takes the stored choice and timings without timing (from_cache
    1) and computes the same pressures bit for bit; a batch of another size
    bucket times its own; a fixed smoother form bypasses the cache (-1)."""
    from paper_1705_05783_amd.batch import Batch
    Batch.clear_tuning_cache()
    pbs = _instances(MIXED_FP32, rtol=1e-8)
    b1, s1, _, p1 = _run_batch(torch, pbs)
    t1 = b1.tuning()
    b1.close()
    b2, s2, _, p2 = _run_batch(torch, pbs)
    t2 = b2.tuning()
    b2.close()
    log("measured", t1, "cached", t2)
    assert t1["from_cache"] == 0 and t2["from_cache"] == 1
    assert {k: v for k, v in t2.items() if k != "from_cache"} == {k: v for k, v in t1.items() if k != "from_cache"}
    assert s1 == s2 and all(s == 0 for s in s1)
    for a, c in zip(p1, p2):
        assert np.array_equal(a, c)
    b3, s3, _, _ = _run_batch(torch, pbs[:2])
    assert b3.tuning()["from_cache"] == 0
    b3.close()
    b4 = Batch.from_problems(pbs)
    b4.set_smoother(256, 1)
    pn = [torch.as_tensor(_start(pb), device="cuda") for pb in pbs]
    p = [t.clone() for t in pn]
    b4.newton_iteration(pn, p)
    assert b4.tuning()["from_cache"] == -1
    b4.close()


def test_batch_of_one_and_iteration_limit(torch):
    """A batch of one instance; an instance that reaches lin_maxit reports
    CAMS_E_NOT_CONVERGED while the others finish."""
    from paper_1705_05783_amd import _cams as C
    pbs = _instances(FP64, rtol=1e-8)[:3]
    b, status, stats, _ = _run_batch(torch, pbs[:1])
    assert status == [0]
    b.close()
    pbs[1] = pbs[1].with_options(lin_maxit=2)
    b, status, stats, _ = _run_batch(torch, pbs)
    log("limit", status, [s["lin_iters_last"] for s in stats])
    assert status[0] == 0 and status[2] == 0
    assert status[1] == C.CAMS_E_NOT_CONVERGED and stats[1]["lin_iters_last"] == 2
    b.close()


def test_batch_full_size_256_instances(torch):
    """The 256-instance uneven batch (mixed precision, one Newton iteration):
    every instance's update meets the linear tolerance on the oracle's own
    FP64 matrix, and sampled instances match the single-problem path."""
    from paper_1705_05783_amd.solver import Solver
    pbs = batch_problems()
    log("cells", sum(pb.n for pb in pbs))
    b, status, stats, p = _run_batch(torch, pbs)
    its = [s["lin_iters_last"] for s in stats]
    log("status", set(status), "iters min/max", min(its), max(its), "tuning", b.tuning(),
        "setup ms", stats[0]["t_coarse_ms"], "iterate ms", stats[0]["t_iterate_ms"])
    assert all(s == 0 for s in status)
    for i, pb in enumerate(pbs):
        T = oracle.transmissibility(pb)
        p0 = _start(pb)
        rel, bound = linear_residual_check(pb, T, p0, p0, p[i])
        assert rel <= bound, (pb.name, rel, bound)
    order = np.argsort([pb.n for pb in pbs])
    for i in (order[0], order[len(order) // 2], order[-1]):
        pb = pbs[i]
        sv = Solver(pb)
        pn = torch.as_tensor(_start(pb), device="cuda")
        ps = pn.clone()
        single = sv.newton_step(pn, ps, check=False)
        diff = rel_err(p[i], to_np(ps))
        log(pb.name, "diff vs single", diff)
        assert diff <= 1e-12 and single["lin_iters_total"] == its[i]
        sv.close()
    b.close()


def test_block_tridiagonal_instance_needs_its_own_factorisation_after_a_batch(torch):
    """The batch inverts every MSFE instance densely; an instance whose own
    coarse solve is block tridiagonal (over 4096 nodes, here 5760) must not
    reuse that inverse: cams_iterate after the batch reports CAMS_E_STATE,
    and after cams_coarse_op the solve meets the tolerance on the oracle's
    matrix."""
    import ctypes
    from paper_1705_05783_amd import _cams as C
    from tests.gpu_util import linear_residual_check
    big = small_problem(96, 96, 40, 4, sigma=2.0, seed=31, c=0.1).with_options(precision=MIXED_FP32, newton_maxit=1)
    small = small_problem(16, 12, 8, 4, sigma=2.0, seed=3, c=0.1).with_options(precision=MIXED_FP32, newton_maxit=1)
    b, status, stats, p = _run_batch(torch, [big, small])
    assert all(s_ == 0 for s_ in status)
    s = b.solvers[0]
    assert C.cams_coarse_planes(s.ctx) > 0
    p0 = _start(big)
    pt = torch.as_tensor(p0, device="cuda")
    s.assemble(pt, pt.clone())
    rc = C.cams_iterate(s.ctx, ctypes.c_void_p(pt.data_ptr()), None)
    assert rc == C.CAMS_E_STATE
    s.coarse_op()
    d = torch.zeros_like(pt)
    s.iterate(d)
    rel, bound = linear_residual_check(big, oracle.transmissibility(big), p0, p0, p0 + to_np(d), d=to_np(d))
    assert rel <= bound, (rel, bound)
    b.close()


def test_mixed_instance_iterates_on_the_batched_inverse_then_on_its_own_rounded_copy(torch):
    """A mixed-precision MSFE instance with a dense inverse above 1024 coarse
    nodes (here 2048) solves alone from an FP32 copy of its inverse; the
    batch rewrites the inverse without rounding it, so cams_iterate on the
    system the batch assembled (at the same start pressure) reads the FP64
    inverse, and after a new assembly and cams_coarse_op the fresh FP32
    copy.  Both solves meet the tolerance on the oracle's matrix."""
    big = small_problem(64, 64, 32, 4, sigma=2.0, seed=33, c=0.1).with_options(precision=MIXED_FP32, newton_maxit=1)
    small = small_problem(16, 12, 8, 4, sigma=2.0, seed=3, c=0.1).with_options(precision=MIXED_FP32, newton_maxit=1)
    b, status, stats, p = _run_batch(torch, [big, small])
    assert all(s_ == 0 for s_ in status)
    s = b.solvers[0]
    assert s.Nc == 2048
    from paper_1705_05783_amd import _cams as C
    assert C.cams_coarse_planes(s.ctx) == 0
    p0 = _start(big)
    T = oracle.transmissibility(big)
    for refactor in (False, True):
        pt = torch.as_tensor(p0, device="cuda")
        if refactor:
            s.assemble(pt, pt.clone())
            s.coarse_op()
        d = torch.zeros_like(pt)
        st = s.iterate(d)
        rel, bound = linear_residual_check(big, T, p0, p0, p0 + to_np(d), d=to_np(d))
        log("refactor", refactor, "iters", st["lin_iters_last"], "relres", rel, "bound", bound)
        assert rel <= bound, (refactor, rel, bound)
    b.close()
