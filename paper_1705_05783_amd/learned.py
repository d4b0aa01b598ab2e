"""Training and use of the learned-basis network (libcams kernels only).

The network (see include/cams.h) predicts the interior basis values of full
dual blocks from their log-transmissibility patch.  Training data are the
exact B4 bases of seeded 64^3 log-normal realisations, built by libcams on
the GPU; the loss, gradients and Adam steps are libcams kernels.  Torch only
holds the device tensors.
"""

from __future__ import annotations

import ctypes
import time

import numpy as np
import torch

from . import _cams as C
from .solver import Solver


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def num_params() -> int:
    return int(C.cams_cnn_num_params())


LAYERS = [(3, 32), (32, 32), (32, 32), (32, 8)]


def init_params(seed: int, device="cuda:0") -> torch.Tensor:
    """He-normal weights (per layer std sqrt(2 / (27 Ci))), zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co in LAYERS:
        parts.append(rng.normal(0.0, np.sqrt(2.0 / (27 * ci)), size=27 * ci * co))
        parts.append(np.zeros(co))
    return torch.tensor(np.concatenate(parts), dtype=torch.float32, device=device)


class Trainer:
    """Adam on the libcams loss/gradient kernels."""

    def __init__(self, params: torch.Tensor, batch: int, lr=1e-3, betas=(0.9, 0.999), eps=1e-8):
        self.params = params
        self.batch = batch
        self.lr, self.betas, self.eps = lr, betas, eps
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.grad = torch.zeros_like(params)
        self.loss = torch.zeros(1, dtype=torch.float64, device=params.device)
        self.ws = torch.empty(int(C.cams_cnn_workspace_bytes(batch)) // 4 + 64, dtype=torch.float32,
                              device=params.device)
        self.t = 0
        self.stream = torch.cuda.current_stream(params.device).cuda_stream

    def loss_grad(self, feat, tgt):
        b = feat.shape[0]
        if b > self.batch:
            raise ValueError("batch larger than the trainer's workspace")
        feat, tgt = feat.contiguous(), tgt.contiguous()
        C.check(C.cams_cnn_loss_grad(ctypes.c_void_p(self.stream), _p(self.params), _p(feat), _p(tgt), b,
                                     _p(self.ws), _p(self.grad), _p(self.loss)), None, "cams_cnn_loss_grad")
        return self.loss, self.grad

    def step(self, feat, tgt):
        self.loss_grad(feat, tgt)
        self.t += 1
        C.check(C.cams_cnn_adam(ctypes.c_void_p(self.stream), _p(self.params), _p(self.grad), _p(self.m),
                                _p(self.v), self.params.numel(), self.t, self.lr, self.betas[0], self.betas[1],
                                self.eps), None, "cams_cnn_adam")
        return self.loss


def forward(params, feat, ws=None, bf16=False):
    """phi (B, 8, 729) of the network; bf16=True: the matrix-core inference
    path the basis construction uses."""
    b = feat.shape[0]
    feat = feat.contiguous()
    phi = torch.empty((b, 8, 729), dtype=torch.float32, device=feat.device)
    stream = torch.cuda.current_stream(feat.device).cuda_stream
    if bf16:
        if ws is None:
            ws = torch.empty(int(C.cams_cnn_bf16_workspace_bytes()) // 4 + 64, dtype=torch.float32,
                             device=feat.device)
        C.check(C.cams_cnn_forward_bf16(ctypes.c_void_p(stream), _p(params), _p(feat), b, _p(ws), _p(phi)), None,
                "cams_cnn_forward_bf16")
        return phi
    if ws is None:
        ws = torch.empty(int(C.cams_cnn_workspace_bytes(b)) // 4 + 64, dtype=torch.float32, device=feat.device)
    C.check(C.cams_cnn_forward(ctypes.c_void_p(stream), _p(params), _p(feat), b, _p(ws), _p(phi)), None,
            "cams_cnn_forward")
    return phi


def training_problem(index: int, seed0: int = 1000):
    """Seeded 64^3 log-normal realisation: sigma ~ U[1,3], correlation length
    ~ U[4,16] cells, ratio 8."""
    from workloads import lognormal_permeability, Problem
    rng = np.random.default_rng(seed0 + index)
    sigma = float(rng.uniform(1.0, 3.0))
    ell = float(rng.uniform(4.0, 16.0))
    n = 64
    perm = lognormal_permeability((n, n, n), 0.0, sigma, ell, seed=seed0 + index).reshape(-1)
    return Problem(f"train{index}", n, n, n, 8, 8, 8, perm, np.full(n ** 3, 0.2), [], c=0.1)


def generate(count: int, seed0: int = 1000, device="cuda:0", log=None):
    """Features and exact targets of the full dual blocks of `count`
    realisations (343 blocks each)."""
    feats, tgts = [], []
    t0 = time.time()
    for i in range(count):
        s = Solver(training_problem(i, seed0), device=device)
        s.build_basis()
        f, t = s.cnn_patches()
        feats.append(f)
        tgts.append(t)
        s.close()
        if log and (i + 1) % max(1, count // 10) == 0:
            log(f"generated {i + 1}/{count} realisations ({time.time() - t0:.1f} s)")
    return torch.cat(feats), torch.cat(tgts)


def train(feat, tgt, epochs=3, batch=256, lr=1e-3, seed=0, log=None, time_limit=None):
    """Adam over shuffled minibatches; returns (params, loss history)."""
    params = init_params(seed, device=feat.device)
    tr = Trainer(params, batch, lr=lr)
    n = feat.shape[0]
    gen = torch.Generator(device="cpu").manual_seed(seed)
    hist = []
    t0 = time.time()
    for ep in range(epochs):
        perm = torch.randperm(n, generator=gen).to(feat.device)
        tot, cnt = 0.0, 0
        for b0 in range(0, n - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            loss = tr.step(feat[idx].contiguous(), tgt[idx].contiguous())
            if cnt % 50 == 0:
                tot += float(loss)
            cnt += 1
            if time_limit and time.time() - t0 > time_limit:
                break
        hist.append(tot / max(1, (cnt + 49) // 50))
        if log:
            log(f"epoch {ep + 1}: mean sampled loss {hist[-1]:.3e} ({time.time() - t0:.1f} s)")
        if time_limit and time.time() - t0 > time_limit:
            break
    return params, hist


def evaluate(params, feat, tgt, batch=256):
    """Mean loss of `params` over all patches (no update)."""
    tr = Trainer(params, batch)
    tot, n = 0.0, feat.shape[0]
    for b0 in range(0, n, batch):
        b = min(batch, n - b0)
        loss, _ = tr.loss_grad(feat[b0:b0 + b], tgt[b0:b0 + b])
        tot += float(loss) * b
    return tot / max(1, n)

