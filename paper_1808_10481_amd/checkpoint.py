"""Checkpoint and resume of a Hermite-leapfrog state.

The state after n steps is (P^n, U^{n+1/2}) plus the plan that defines the
step (d, m, cells, box, dt, c, precision, boundary).  A checkpoint is the two
device buffers copied byte for byte (the library's device layout, which is
fixed by those plan parameters) and a JSON header holding the parameters,
the step count, the byte sizes and a SHA-256 of each buffer.  Restoring
copies the bytes back, so a resumed run continues bit for bit where the
saved one stopped (the step is deterministic).

Files: <prefix>.json, <prefix>.p.bin, <prefix>.u.bin.
"""

from __future__ import annotations

import hashlib
import json
import os

import numpy as np

FORMAT = "hermite-leapfrog-state/1"


def _plan_params(plan) -> dict:
    pr = plan.problem
    return {"d": plan.d, "m": plan.m, "cells": list(plan.cells),
            "length": [float(pr.length[k]) for k in range(plan.d)],
            "dt": float(plan.dt), "c": float(pr.c), "precision": plan.precision,
            "boundary": plan.boundary,
            "p_words": int(plan.info.p_words), "u_words": int(plan.info.u_words),
            "word_bytes": int(plan.info.word_bytes)}


def _host_bytes(t) -> bytes:
    return t.detach().contiguous().cpu().numpy().tobytes()


def save(plan, p, u, step: int, prefix: str) -> dict:
    """Write the state (p, u) of `plan` after `step` steps.  Synchronous."""
    params = _plan_params(plan)
    blobs = {}
    for name, t, words in (("p", p, params["p_words"]), ("u", u, params["u_words"])):
        b = _host_bytes(t)
        if len(b) != words * params["word_bytes"]:
            raise ValueError(f"{name}: {len(b)} bytes, the plan's layout has {words * params['word_bytes']}")
        blobs[name] = b
    header = {"format": FORMAT, "step": int(step), "plan": params,
              "sha256": {k: hashlib.sha256(v).hexdigest() for k, v in blobs.items()}}
    d = os.path.dirname(os.path.abspath(prefix))
    os.makedirs(d, exist_ok=True)
    for k, v in blobs.items():
        with open(f"{prefix}.{k}.bin", "wb") as f:
            f.write(v)
    with open(f"{prefix}.json", "w") as f:
        json.dump(header, f, indent=1)
    return header


def read_header(prefix: str) -> dict:
    with open(f"{prefix}.json") as f:
        h = json.load(f)
    if h.get("format") != FORMAT:
        raise ValueError(f"{prefix}.json: not a {FORMAT} checkpoint")
    return h


def make_plan(header: dict):
    """A plan with the checkpoint's parameters."""
    from paper_1808_10481_amd import hl
    q = header["plan"]
    return hl.Plan(q["d"], q["m"], q["cells"], length=q["length"], dt=q["dt"], c=q["c"],
                   precision=q["precision"], boundary=q["boundary"])


def restore(plan, p, u, prefix: str) -> int:
    """Copy a checkpoint into the device buffers (p, u) of a plan with the
    same parameters; returns the step count.  Raises ValueError on a
    parameter mismatch or a corrupted buffer.  Synchronous."""
    import torch
    h = read_header(prefix)
    want = _plan_params(plan)
    for k, v in want.items():
        got = h["plan"].get(k)
        if k in ("length", "dt", "c"):
            if not np.allclose(got, v, rtol=0, atol=0):
                raise ValueError(f"checkpoint {k} = {got}, plan has {v}")
        elif got != v:
            raise ValueError(f"checkpoint {k} = {got}, plan has {v}")
    for name, t in (("p", p), ("u", u)):
        with open(f"{prefix}.{name}.bin", "rb") as f:
            b = f.read()
        if hashlib.sha256(b).hexdigest() != h["sha256"][name]:
            raise ValueError(f"{prefix}.{name}.bin: checksum mismatch")
        if len(b) != t.numel() * t.element_size():
            raise ValueError(f"{name}: {len(b)} bytes in the file, buffer holds {t.numel() * t.element_size()}")
        host = torch.frombuffer(bytearray(b), dtype=t.dtype)
        t.view(-1).copy_(host.to(t.device))
    if p.is_cuda:
        torch.cuda.synchronize(p.device)
    return int(h["step"])
