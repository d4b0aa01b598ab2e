"""Learned basis on the GPU: the network's forward, loss gradient and Adam
kernels against the FP64 oracle (FP32 kernels: 1e-5 relative), patch
extraction against the oracle basis, and the learned build with fallback."""

import numpy as np
import pytest

import oracle
from oracle import cnn as ocnn
from tests.gpu_util import checked_newton_step, log, rel_err, require_gpu, solver_for, to_np
from workloads import small_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _rand_params(seed):
    p = ocnn.init_params(seed)
    rng = np.random.default_rng(seed + 1)
    # non-zero biases so their gradients are exercised
    o = 0
    for ci, co in ocnn.LAYERS:
        o += 27 * ci * co
        p[o:o + co] = rng.normal(0, 0.1, co)
        o += co
    return p


def test_forward_matches_oracle(torch):
    from paper_1705_05783_amd import learned
    rng = np.random.default_rng(0)
    params = _rand_params(1)
    feat = rng.normal(size=(3, 3, 9, 9, 9))
    phi_ref, _ = ocnn.forward(params, feat)
    pt = torch.tensor(params, dtype=torch.float32, device="cuda")
    ft = torch.tensor(feat.reshape(3, 3, 729), dtype=torch.float32, device="cuda")
    phi = to_np(learned.forward(pt, ft)).reshape(3, 8, 9, 9, 9)
    assert rel_err(phi, phi_ref) <= 2e-5


def test_forward_bf16_matches_oracle(torch):
    """Matrix-core inference (BF16 weights and activations, FP32 accumulation)
    against the FP64 oracle: bfloat16 keeps 8 significant bits, so the basis
    values (in [0, 1]) agree to 0.03 in the worst cell and 3e-3 on average."""
    from paper_1705_05783_amd import learned
    rng = np.random.default_rng(10)
    params = _rand_params(11)
    feat = rng.normal(size=(5, 3, 9, 9, 9))
    phi_ref, _ = ocnn.forward(params, feat)
    pt = torch.tensor(params, dtype=torch.float32, device="cuda")
    ft = torch.tensor(feat.reshape(5, 3, 729), dtype=torch.float32, device="cuda")
    phi = to_np(learned.forward(pt, ft, bf16=True)).reshape(5, 8, 9, 9, 9)
    d = np.abs(phi - phi_ref)
    log("bf16 inference: max", d.max(), "mean", d.mean())
    assert d.max() <= 0.03 and d.mean() <= 3e-3
    assert np.allclose(phi.sum(axis=1), 1.0, atol=1e-5)


def test_loss_gradient_matches_oracle(torch):
    from paper_1705_05783_amd import learned
    rng = np.random.default_rng(2)
    params = _rand_params(3)
    feat = rng.normal(size=(5, 3, 9, 9, 9))
    tgt = rng.dirichlet(np.ones(8), size=(5, 7, 7, 7)).transpose(0, 4, 1, 2, 3)
    loss_ref, g_ref = ocnn.loss_and_grad(params, feat, tgt)
    pt = torch.tensor(params, dtype=torch.float32, device="cuda")
    tr = learned.Trainer(pt, batch=5)
    loss, g = tr.loss_grad(torch.tensor(feat.reshape(5, 3, 729), dtype=torch.float32, device="cuda"),
                           torch.tensor(tgt.reshape(5, 8, 343), dtype=torch.float32, device="cuda"))
    log("loss", float(loss), loss_ref)
    assert abs(float(loss) - loss_ref) <= 1e-5 * loss_ref
    g = to_np(g).astype(np.float64)
    o = 0
    for ci, co in ocnn.LAYERS:
        n = 27 * ci * co + co
        assert rel_err(g[o:o + n], g_ref[o:o + n]) <= 1e-4, (ci, co)
        o += n


def test_adam_matches_oracle(torch):
    from paper_1705_05783_amd import learned
    rng = np.random.default_rng(4)
    n = learned.num_params()
    p0 = rng.normal(size=n)
    pt = torch.tensor(p0, dtype=torch.float32, device="cuda")
    tr = learned.Trainer(pt, batch=1, lr=1e-2)
    p, m, v = p0.astype(np.float32).astype(np.float64), np.zeros(n), np.zeros(n)
    import ctypes
    from paper_1705_05783_amd import _cams as C
    for t in range(1, 4):
        g = rng.normal(size=n)
        tr.grad.copy_(torch.tensor(g, dtype=torch.float32))
        C.cams_cnn_adam(ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), ctypes.c_void_p(pt.data_ptr()),
                        ctypes.c_void_p(tr.grad.data_ptr()), ctypes.c_void_p(tr.m.data_ptr()),
                        ctypes.c_void_p(tr.v.data_ptr()), n, t, 1e-2, 0.9, 0.999, 1e-8)
        p, m, v = ocnn.adam_step(p, g.astype(np.float32).astype(np.float64), m, v, t, lr=1e-2)
    torch.cuda.synchronize()
    assert rel_err(to_np(pt), p) <= 1e-5


def _learned_problem():
    return small_problem(26, 24, 20, 8, sigma=2.0, seed=21)


def test_patches_match_oracle_basis(torch):
    pb = _learned_problem()
    s = solver_for(pb)
    s.build_basis()
    feat, tgt = s.cnn_patches()
    nb = feat.shape[0]
    assert nb == s.num_full_blocks() and nb > 0
    T = oracle.transmissibility(pb)
    P = oracle.basis_b4(pb, T)
    v = [list(oracle.vertex_coords(n, 8)) for n in (pb.nx, pb.ny, pb.nz)]
    blocks = [(a, b, c) for c in range(len(v[2]) - 1) for b in range(len(v[1]) - 1) for a in range(len(v[0]) - 1)
              if v[0][a + 1] - v[0][a] == 8 and v[1][b + 1] - v[1][b] == 8 and v[2][c + 1] - v[2][c] == 8]
    assert len(blocks) == nb
    F = to_np(feat).reshape(nb, 3, 9, 9, 9)
    G = to_np(tgt).reshape(nb, 8, 7, 7, 7)
    Tg = T.reshape(3, pb.nz, pb.ny, pb.nx)
    Pg = P.reshape(8, pb.nz, pb.ny, pb.nx)
    found = 0
    for (a, b, c) in blocks:
        x0, y0, z0 = v[0][a], v[1][b], v[2][c]
        ref_t = Pg[:, z0 + 1:z0 + 8, y0 + 1:y0 + 8, x0 + 1:x0 + 8]
        # locate this block among the GPU patches by its targets
        k = int(np.argmin([np.abs(G[q] - ref_t).max() for q in range(nb)]))
        assert np.abs(G[k] - ref_t).max() <= 1e-6
        lnT = np.log(np.where(Tg > 0, Tg, 1.0))[:, z0:z0 + 9, y0:y0 + 9, x0:x0 + 9].copy()
        lnT[0, :, :, 8] = 0
        lnT[1, :, 8, :] = 0
        lnT[2, 8, :, :] = 0
        assert np.abs(F[k] - lnT).max() <= 1e-5 * max(1.0, np.abs(lnT).max())
        found += 1
    assert found == nb


def test_learned_build_fallback_and_prediction(torch):
    """Tiny tolerance: every predicted block falls back, the basis is exact.
    Huge tolerance: interiors are the network's softmax output (partition of
    unity), and the Newton step still converges to the oracle pressure."""
    from paper_1705_05783_amd import learned
    pb = _learned_problem()
    params = torch.tensor(_rand_params(7), dtype=torch.float32, device="cuda")
    T = oracle.transmissibility(pb)
    P_ref = oracle.basis_b4(pb, T)
    s = solver_for(pb)
    s.set_learned(params, fallback_tol=1e-12)
    s.build_basis()
    st = s.basis_stats()
    assert st["fallback_blocks"] == s.num_full_blocks() and st["learned_blocks"] == 0
    assert np.max(np.abs(to_np(s.export(4)).reshape(8, -1) - P_ref)) <= 1e-12

    s2 = solver_for(pb)
    s2.set_learned(params, fallback_tol=1e30)
    s2.build_basis()
    st2 = s2.basis_stats()
    assert st2["learned_blocks"] == s2.num_full_blocks() and st2["fallback_blocks"] == 0
    P = to_np(s2.export(4)).reshape(8, -1)
    assert np.max(np.abs(P.sum(axis=0) - 1.0)) <= 1e-5
    feat, _ = s2.cnn_patches(with_targets=False)
    phi = to_np(learned.forward(params, feat, bf16=True)).reshape(-1, 8, 9, 9, 9)
    # every predicted interior appears in the basis
    Pg = P.reshape(8, pb.nz, pb.ny, pb.nx)
    v = [list(oracle.vertex_coords(n, 8)) for n in (pb.nx, pb.ny, pb.nz)]
    x0, y0, z0 = v[0][0], v[1][0], v[2][0]
    block = Pg[:, z0 + 1:z0 + 8, y0 + 1:y0 + 8, x0 + 1:x0 + 8]
    assert min(np.abs(phi[q][:, 1:8, 1:8, 1:8] - block).max() for q in range(phi.shape[0])) <= 1e-6
    pn = pb.initial_pressure()
    p = torch.as_tensor(pn, device="cuda")
    s2.newton_step(p.clone(), p)
    _, e = oracle.nonlinear_residual(pb, T, to_np(p), pn)
    assert e <= pb.newton_tol
    p_ref, rc, _ = oracle.newton_step(pb, T, P_ref, pn, pn)
    assert rel_err(to_np(p), p_ref) <= 1e-6


def test_short_training_reduces_loss(torch):
    from paper_1705_05783_amd import learned
    feat, tgt = learned.generate(2, seed0=4000)
    assert feat.shape == (2 * 343, 3, 729)
    params, hist = learned.train(feat, tgt, epochs=3, batch=64, lr=2e-3, seed=1)
    log("loss history", hist)
    assert hist[-1] < hist[0]


def test_trained_network_gain(torch):
    """What the trained network brings, on the 128^3 evaluation field (a seed
    outside the training set): against exact local solves its basis error is
    far below that of the untrained network, and the C-AMS iterations of one
    time step with its basis (no fallback) stay within 10% of the exact
    basis, while the untrained network's basis needs more."""
    from paper_1705_05783_amd import _cams as C
    from paper_1705_05783_amd import learned
    from paper_1705_05783_amd.solver import Solver
    from paper_1705_05783_amd.train_basis import load_weights
    from workloads.configs import FP64, MIXED_FP32, config5_eval

    trained = load_weights()
    untrained = learned.init_params(0)
    pb = config5_eval(precision=FP64)
    s = Solver(pb)
    s.build_basis()
    P_exact = s.export(C.CAMS_ARR_P)
    err = {}
    for name, params in (("trained", trained), ("untrained", untrained)):
        s.set_learned(params, fallback_tol=1e30)
        s.build_basis()
        err[name] = float((s.export(C.CAMS_ARR_P) - P_exact).norm() / P_exact.norm())
    s.close()
    iters = {}
    for name, params in (("exact", None), ("trained", trained), ("untrained", untrained)):
        pbm = config5_eval(precision=MIXED_FP32)
        sm = Solver(pbm)
        if params is not None:
            sm.set_learned(params, fallback_tol=1e30)
        pn = sm.new_pressure()
        p = pn.clone()
        st = sm.newton_step(pn, p, check=False)
        iters[name] = st["lin_iters_total"] if st["status"] == 0 else 10 ** 9
        sm.close()
    log("basis rel. L2 error", err, "C-AMS iterations (one time step)", iters)
    assert err["trained"] < 0.5 * err["untrained"]
    assert iters["trained"] <= 1.1 * iters["exact"]
    assert iters["untrained"] > iters["trained"]


def test_fallback_at_an_intermediate_tolerance(torch):
    """The per-block guard where it acts on some blocks and not others.  With
    the trained network and no fallback, the GPU's ratio of every full dual
    block matches the oracle's recomputation from the exported basis.  Then,
    with fallback_tol between two ratios near the median, exactly the blocks
    above it are re-solved: their interiors equal the oracle's exact basis
    (1e-12), the others keep the network's values bit for bit, and every
    other cell is exact."""
    from paper_1705_05783_amd import _cams as C
    from paper_1705_05783_amd.train_basis import load_weights
    pb = small_problem(64, 64, 32, 8, sigma=2.5, seed=23)
    params = load_weights()
    T = oracle.transmissibility(pb)
    P_ref = oracle.basis_b4(pb, T)
    starts = oracle.full_dual_blocks(pb)
    s = solver_for(pb)
    nb = s.num_full_blocks()
    assert nb == len(starts) == 147
    s.set_learned(params, fallback_tol=1e30)
    s.build_basis()
    P_net = to_np(s.export(C.CAMS_ARR_P)).reshape(8, -1)
    r_gpu = s.block_ratios()
    r_ref = oracle.basis_block_ratios(pb, T, P_net, starts)
    log("ratios: min", r_ref.min(), "median", np.median(r_ref), "max", r_ref.max(),
        "gpu vs oracle", rel_err(r_gpu, r_ref))
    assert rel_err(r_gpu, r_ref) <= 1e-12
    order = np.sort(r_ref)
    k = nb // 2
    tol = 0.5 * (order[k - 1] + order[k])
    assert order[k] - order[k - 1] > 1e-9 * tol      # no block sits at the threshold
    above = r_ref > tol
    s.set_learned(params, fallback_tol=tol)
    s.build_basis()
    st = s.basis_stats()
    log("fallback_tol", tol, st)
    assert st["fallback_blocks"] == int(above.sum()) and st["learned_blocks"] == nb - int(above.sum())
    P_fb = to_np(s.export(C.CAMS_ARR_P)).reshape(8, pb.nz, pb.ny, pb.nx)
    Pn = P_net.reshape(8, pb.nz, pb.ny, pb.nx)
    Pr = P_ref.reshape(8, pb.nz, pb.ny, pb.nx)
    interior = np.zeros((pb.nz, pb.ny, pb.nx), dtype=bool)
    for b, (x0, y0, z0) in enumerate(starts):
        sl = (slice(None), slice(z0, z0 + 7), slice(y0, y0 + 7), slice(x0, x0 + 7))
        interior[sl[1:]] = True
        if above[b]:
            assert np.max(np.abs(P_fb[sl] - Pr[sl])) <= 1e-12, b
        else:
            assert np.array_equal(P_fb[sl], Pn[sl]), b
    assert np.max(np.abs(P_fb[:, ~interior] - Pr[:, ~interior])) <= 1e-12
    # the stats of a Newton step report the same count
    pn = torch.as_tensor(pb.initial_pressure(), device="cuda")
    s.invalidate_basis()
    st2 = s.newton_step(pn.clone(), pn.clone())
    assert st2["fallback_blocks"] == int(above.sum())
    s.close()


def test_config5_learned_mixed_full_size(torch):
    """The metric's learned+mixed configuration at full size: 128^3 (seed 5,
    outside the network's training seeds), trained network for the full
    dual-block interiors with the calibrated fallback tolerance, FP32 basis
    storage and smoother, FP64 refinement.  One time step through the ABI's
    hot-path calls: every linear solve meets 1e-8 on the oracle's own FP64
    matrix, and the oracle's nonlinear error of the GPU pressure meets the
    Newton tolerance."""
    from paper_1705_05783_amd.train_basis import load_fallback_tol, load_weights
    from workloads.configs import config5_eval
    pb = config5_eval()
    s = solver_for(pb)
    s.set_learned(load_weights(), fallback_tol=load_fallback_tol())
    T = oracle.transmissibility(pb)
    pn_t = torch.as_tensor(pb.initial_pressure(), device="cuda")
    p_t = pn_t.clone()
    nit, lits, worst = checked_newton_step(s, pb, T, pn_t, p_t, torch)
    _, e = oracle.nonlinear_residual(pb, T, to_np(p_t), to_np(pn_t))
    log("128^3 learned+mixed: newton", nit, "cams", lits, "worst relres/bound", worst, "eps", e,
        s.basis_stats())
    assert nit >= 1 and e <= pb.newton_tol
    s.close()


def test_learned_global_guard(torch):
    """The global check of the learned basis (cams_set_learned_guard).  On a
    64x64x32 field the exact basis needs n_plain C-AMS iterations per solve.
    With the trained network, the calibrated per-block fallback and the check
    at n_plain, no rebuild happens (the network's solves stay well below
    twice that).  With the check at one iteration, which every learned solve
    exceeds, the first solve triggers it: afterwards the basis equals the
    oracle's exact basis (local solves), the time step still converges (the
    oracle's nonlinear error of the pressure meets the Newton tolerance), and
    the next time step, already on the exact basis, rebuilds nothing.  A
    negative count is refused."""
    from paper_1705_05783_amd import _cams as C
    from paper_1705_05783_amd.train_basis import load_fallback_tol, load_weights
    pb = small_problem(64, 64, 32, 8, sigma=2.5, seed=23)
    T = oracle.transmissibility(pb)
    pn = torch.as_tensor(pb.initial_pressure(), device="cuda")
    exact = solver_for(pb)
    st0 = exact.newton_step(pn.clone(), pn.clone())
    plain = -(-st0["lin_iters_total"] // st0["newton_iters"])
    exact.close()
    params = load_weights()
    s = solver_for(pb)
    s.set_learned(params, fallback_tol=load_fallback_tol(), guard_iters=plain)
    st1 = s.newton_step(pn.clone(), pn.clone())
    log("exact basis: C-AMS per solve", plain, "| learned with the check at that count:", st1["lin_iters_total"],
        "over", st1["newton_iters"], "solves, rebuilds", st1["basis_rebuilds"])
    assert st1["basis_rebuilds"] == 0
    s.close()
    s = solver_for(pb)
    s.set_learned(params, fallback_tol=load_fallback_tol(), guard_iters=1)
    p = pn.clone()
    st2 = s.newton_step(pn.clone(), p)
    log("check at one iteration:", st2)
    assert st2["basis_rebuilds"] == 1
    P = to_np(s.export(C.CAMS_ARR_P)).reshape(8, -1)
    assert np.max(np.abs(P - oracle.basis_b4(pb, T))) <= 1e-12
    _, e = oracle.nonlinear_residual(pb, T, to_np(p), to_np(pn))
    assert e <= pb.newton_tol
    st3 = s.newton_step(p.clone(), p.clone())
    assert st3["basis_rebuilds"] == 0
    assert C.cams_set_learned_guard(s.ctx, -1) == C.CAMS_E_ARG
    s.close()
