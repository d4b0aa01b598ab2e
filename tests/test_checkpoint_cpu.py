"""Checkpoint format on the CPU (no GPU, no basis): a save/load round trip
returns the pressure, step and time unchanged; a checkpoint is refused by a
solver of another problem, when an array is damaged, and when the manifest
is missing (an interrupted save)."""

import os
import types

import numpy as np
import pytest
import torch

from paper_1705_05783_amd import checkpoint
from workloads import small_problem


def _stub(pb):
    opts = types.SimpleNamespace(restriction=1, n_pre=0, n_post=5, precision=0, smoother=2, basis_type=0)
    return types.SimpleNamespace(pb=pb, options=opts, device=torch.device("cpu"), N=pb.n)


def test_round_trip_and_refusals(tmp_path):
    pb = small_problem(12, 10, 6, 3, sigma=1.5, seed=4)
    s = _stub(pb)
    p = torch.as_tensor(np.random.default_rng(1).uniform(0, 1, pb.n))
    d = str(tmp_path / "ck")
    checkpoint.save(s, d, p, 7, 0.35, with_basis=False)
    q, step, t = checkpoint.load(s, d)
    assert torch.equal(q, p) and step == 7 and t == 0.35
    other = _stub(pb.with_options(dt=pb.dt * 2))
    with pytest.raises(ValueError, match="fluid"):
        checkpoint.load(other, d)
    rock = _stub(small_problem(12, 10, 6, 3, sigma=1.5, seed=5))
    with pytest.raises(ValueError, match="perm"):
        checkpoint.load(rock, d)
    raw = bytearray(open(os.path.join(d, "pressure.f64"), "rb").read())
    raw[17] ^= 1
    open(os.path.join(d, "pressure.f64"), "wb").write(bytes(raw))
    with pytest.raises(ValueError, match="damaged"):
        checkpoint.load(s, d)
    os.remove(os.path.join(d, "state.json"))
    with pytest.raises(FileNotFoundError):
        checkpoint.load(s, d)
