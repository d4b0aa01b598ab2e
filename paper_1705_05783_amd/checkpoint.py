"""Checkpoint and resume of a time-stepping run.

The state after a completed time step (Sec. 2, backward Euler) is the
pressure p^n that the next step starts from, the step index and the time;
for the basis types B3 and B4 the basis depends on the rock only (Sec. 3),
so it is saved too and a resumed run skips its rebuild.  A checkpoint is a
directory of raw little-endian float64 arrays (``pressure.f64``,
``basis.f64``) and ``state.json``: format tag, step, time, the problem's key
(grid, fluid, solver options and SHA-256 digests of the rock arrays) and,
per array, its length and SHA-256 digest.  Nothing is pickled.  Loading
checks the key against the solver it is loaded into and every digest, and
raises ValueError on any mismatch.
"""

from __future__ import annotations

import hashlib
import json
import os

import numpy as np
import torch

from . import _cams as C

FORMAT = "cams-checkpoint-1"
_OPTION_FIELDS = ("restriction", "n_pre", "n_post", "precision", "smoother", "basis_type")


def _digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<f8").tobytes()).hexdigest()


def problem_key(solver) -> dict:
    """What a checkpoint must agree on with the solver that resumes it."""
    pb = solver.pb
    key = {"grid": [int(pb.nx), int(pb.ny), int(pb.nz), float(pb.dx), float(pb.dy), float(pb.dz),
                    int(pb.rx), int(pb.ry), int(pb.rz)],
           "fluid": [float(pb.rho0), float(pb.c), float(pb.p0), float(pb.mu), float(pb.dt)],
           "options": {f: int(getattr(solver.options, f)) for f in _OPTION_FIELDS},
           "perm_sha256": _digest(pb.perm), "phi_sha256": _digest(pb.phi),
           "wells": [[int(c), float(v)] for c, v in pb.wells]}
    return key


def save(solver, path: str, pn: torch.Tensor, step: int, time: float, with_basis: bool = True) -> None:
    """Write the state after time step `step` (pressure pn at `time`)."""
    os.makedirs(path, exist_ok=True)
    arrays = {"pressure": pn}
    if with_basis:
        if int(solver.options.basis_type) not in (0, 3):
            raise ValueError("only the pressure-independent bases (B3, B4) are saved")
        arrays["basis"] = solver.export(C.CAMS_ARR_P)
    meta = {"format": FORMAT, "step": int(step), "time": float(time), "problem": problem_key(solver),
            "arrays": {}}
    for name, t in arrays.items():
        a = t.detach().to("cpu").contiguous().numpy().astype("<f8", copy=False)
        raw = a.tobytes()
        with open(os.path.join(path, name + ".f64"), "wb") as f:
            f.write(raw)
        meta["arrays"][name] = {"file": name + ".f64", "count": int(a.size),
                                "sha256": hashlib.sha256(raw).hexdigest()}
    tmp = os.path.join(path, "state.json.tmp")
    with open(tmp, "w") as f:
        json.dump(meta, f, indent=1)
    os.replace(tmp, os.path.join(path, "state.json"))   # the manifest appears last


def _read(path: str, spec: dict) -> np.ndarray:
    with open(os.path.join(path, spec["file"]), "rb") as f:
        raw = f.read()
    if len(raw) != 8 * int(spec["count"]) or hashlib.sha256(raw).hexdigest() != spec["sha256"]:
        raise ValueError(f"checkpoint array {spec['file']} is damaged")
    return np.frombuffer(raw, dtype="<f8").astype(np.float64)


def load(solver, path: str):
    """Resume: returns (pn on the solver's device, step, time) and, when the
    checkpoint holds a basis, installs it in the solver."""
    with open(os.path.join(path, "state.json")) as f:
        meta = json.load(f)
    if meta.get("format") != FORMAT:
        raise ValueError(f"not a checkpoint of this format: {meta.get('format')!r}")
    want, have = meta["problem"], problem_key(solver)
    diff = sorted(k for k in set(want) | set(have) if want.get(k) != have.get(k))
    if diff:
        raise ValueError("checkpoint belongs to another problem: " + ", ".join(diff))
    specs = meta["arrays"]
    pn = _read(path, specs["pressure"])
    if pn.size != solver.N:
        raise ValueError("checkpoint pressure has the wrong length")
    pn_t = torch.as_tensor(pn, device=solver.device)
    if "basis" in specs:
        solver.import_basis(torch.as_tensor(_read(path, specs["basis"]), device=solver.device))
    return pn_t, int(meta["step"]), float(meta["time"])
