"""Training driver of the learned-basis network.

    python -m paper_1705_05783_amd.train_basis --count 200 --epochs 8

Builds the exact B4 bases of `count` seeded 64^3 log-normal realisations
with libcams, trains the network on their full dual blocks with the libcams
loss/gradient/Adam kernels, and writes the FP32 parameters (flat, in the
layer order of include/cams.h) plus a JSON record of the run next to this
file.  Needs a GPU.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import learned
from .solver import Solver

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "weights", "cnn_basis_f32.npy")
RECORD = os.path.join(HERE, "weights", "cnn_basis_train.json")


def load_weights(path=WEIGHTS, device="cuda:0") -> torch.Tensor:
    """Trained parameters as a float32 device tensor."""
    arr = np.load(path, allow_pickle=False)
    if arr.dtype != np.float32 or arr.ndim != 1 or arr.size != learned.num_params():
        raise ValueError(f"{path}: expected {learned.num_params()} float32 parameters")
    return torch.tensor(arr, device=device)


def load_fallback_tol(path=RECORD) -> float:
    """The calibrated per-block fallback tolerance of the trained network
    (see `calibrate`)."""
    with open(path) as f:
        rec = json.load(f)
    return float(rec["fallback_tol"]["value"])


def calibrate(params, count, seed0, quantile=0.99, log=None):
    """Per-block local-equation ratios ||(T Phi)_I|| / ||T_IF Phi_F|| of the
    network's interiors on `count` held-out realisations drawn like the
    training set (seeds seed0 .. seed0 + count - 1, past the training and
    validation seeds), with no fallback.  The fallback tolerance is their
    `quantile` quantile: a block whose prediction is worse than the network
    achieves on that share of in-distribution blocks is taken as outside
    what it learned and re-solved exactly.  Returns (tolerance, summary)."""
    ratios = []
    for i in range(count):
        s = Solver(learned.training_problem(i, seed0))
        s.set_learned(params, fallback_tol=1e30)
        s.build_basis()
        ratios.append(s.block_ratios())
        s.close()
        if log:
            log(f"calibration realisation {i + 1}/{count}: median ratio {np.median(ratios[-1]):.3e}")
    r = np.concatenate(ratios)
    q = np.quantile(r, [0.5, 0.9, quantile, 1.0])
    return float(q[2]), {"blocks": int(r.size), "median": float(q[0]), "p90": float(q[1]),
                         "quantile": quantile, "max": float(q[3])}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=200, help="training realisations (343 patches each)")
    ap.add_argument("--holdout", type=int, default=8, help="further realisations for the validation loss")
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch", type=int, default=128)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed0", type=int, default=1000)
    ap.add_argument("--time-limit", type=float, default=None, help="seconds of training")
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--record", default=RECORD)
    ap.add_argument("--calibrate", type=int, default=0, metavar="COUNT",
                    help="only calibrate the fallback tolerance of the stored network on COUNT held-out "
                         "realisations and add it to the record")
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    if a.calibrate:
        with open(a.record) as f:
            rec = json.load(f)
        seed_cal = rec["seed0"] + rec["realisations"] + rec["holdout_realisations"]
        tol, summary = calibrate(load_weights(a.out), a.calibrate, seed_cal, log=log)
        rec["fallback_tol"] = {"value": tol, "seed0": seed_cal, "realisations": a.calibrate, **summary,
                               "command": " ".join(["python -m paper_1705_05783_amd.train_basis"] +
                                                   (argv or sys.argv[1:]))}
        with open(a.record, "w") as f:
            json.dump(rec, f, indent=1)
        log(json.dumps(rec["fallback_tol"]))
        return

    t0 = time.time()
    feat, tgt = learned.generate(a.count, seed0=a.seed0, log=log)
    vfeat, vtgt = learned.generate(a.holdout, seed0=a.seed0 + a.count)
    t_gen = time.time() - t0
    log(f"{feat.shape[0]} training patches, {vfeat.shape[0]} validation patches ({t_gen:.1f} s)")

    t1 = time.time()
    params, hist = learned.train(feat, tgt, epochs=a.epochs, batch=a.batch, lr=a.lr, log=log,
                                 time_limit=a.time_limit)
    torch.cuda.synchronize()
    t_train = time.time() - t1
    vloss = learned.evaluate(params, vfeat, vtgt)
    log(f"validation loss {vloss:.3e}")

    np.save(a.out, params.cpu().numpy().astype(np.float32), allow_pickle=False)
    rec = {"realisations": a.count, "patches": int(feat.shape[0]), "holdout_realisations": a.holdout,
           "seed0": a.seed0, "epochs_run": len(hist), "batch": a.batch, "lr": a.lr,
           "loss_per_epoch": hist, "validation_loss": vloss, "generate_s": t_gen, "train_s": t_train,
           "command": " ".join(["python -m paper_1705_05783_amd.train_basis"] + (argv or sys.argv[1:]))}
    with open(a.record, "w") as f:
        json.dump(rec, f, indent=1)
    log(json.dumps(rec))


if __name__ == "__main__":
    main()
