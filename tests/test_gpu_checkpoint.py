"""Resume from a checkpoint on the GPU: three time steps run through, and
the same run stopped after step 1, saved (with the basis, or without it so
that the resumed solver rebuilds it) and resumed by a fresh solver, end on
the same pressure bit for bit (the kernels are deterministic), in FP64 and
in the mixed precision, where the imported basis is rounded as after a
build."""

import numpy as np
import pytest

from paper_1705_05783_amd import checkpoint
from tests.gpu_util import log, require_gpu, solver_for, to_np
from workloads import small_problem
from workloads.configs import FP64, MIXED_FP32

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _steps(s, pn, p, k):
    for _ in range(k):
        s.newton_step(pn, p)
        pn.copy_(p)


@pytest.mark.parametrize("precision", [FP64, MIXED_FP32])
def test_resume_matches_the_uninterrupted_run(torch, tmp_path, precision):
    pb = small_problem(24, 20, 16, 4, sigma=2.0, seed=9).with_options(precision=precision)
    s = solver_for(pb)
    pn = s.new_pressure()
    p = pn.clone()
    _steps(s, pn, p, 3)
    ref = to_np(p)
    s.close()
    s = solver_for(pb)
    pn = s.new_pressure()
    p = pn.clone()
    _steps(s, pn, p, 1)
    dirs = {True: str(tmp_path / "with_basis"), False: str(tmp_path / "without")}
    for with_basis, d in dirs.items():
        checkpoint.save(s, d, pn, 1, pb.dt, with_basis=with_basis)
    s.close()
    for with_basis, d in dirs.items():
        r = solver_for(pb)
        pn_r, step, t = checkpoint.load(r, d)
        assert step == 1 and t == pb.dt
        p_r = pn_r.clone()
        _steps(r, pn_r, p_r, 3 - step)
        got = to_np(p_r)
        log("precision", precision, "basis saved", with_basis, "max |diff|", float(np.abs(got - ref).max()))
        assert np.array_equal(got, ref)
        r.close()
