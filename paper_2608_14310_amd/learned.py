"""Training loop and checkpoints of the learned correction stage.

Argument marshalling and loop control only: residual pairs come from the
library's V-cycle (`Solver.learned_pairs`), every forward/backward/Adam step
runs in the library's kernels (`Net.train_step`). Random draws (exact
solutions, batch order) are inputs made by the caller.
"""
from __future__ import annotations

import json
import os
from typing import Dict, Iterable, List, Optional

import numpy as np


def generate_pairs(solver, xstar, iters: int = 3, chunk: int = 64):
    """(rhat, ehat) float32 device tensors, one pair per (x*, V-cycle iteration);
    xstar is a float64 device tensor (count, 3N^2), processed in chunks."""
    import torch
    rs, es = [], []
    for k in range(0, int(xstar.shape[0]), chunk):
        r, e = solver.learned_pairs(xstar[k:k + chunk].contiguous(), iters)
        rs.append(r)
        es.append(e)
    return torch.cat(rs), torch.cat(es)


def train(net, rhat, ehat, N: int, batches: Iterable[np.ndarray], lr: float = 1e-3,
          log_every: int = 0, solver=None, kind: str = "residual") -> List[float]:
    """One Adam step per index array in `batches`; returns the loss of each step.
    With `solver` the loss is the residual norm through the solver's K_E
    (ehat unused); otherwise the error loss against ehat."""
    losses = []
    for k, idx in enumerate(batches):
        if solver is not None:
            losses.append(solver.train_net_residual(net, rhat, idx, lr, kind))
        else:
            losses.append(net.train_step(rhat, ehat, N, idx, lr))
        if log_every and (k + 1) % log_every == 0:
            print(f"[train] step {k + 1} loss {np.mean(losses[-log_every:]):.4f}", flush=True)
    return losses


def save_weights(path: str, w: np.ndarray, meta: Optional[Dict] = None) -> None:
    """Checkpoint: the 10 944 master weights as .npy plus a JSON sidecar."""
    np.save(path, np.ascontiguousarray(w, dtype=np.float32), allow_pickle=False)
    with open(os.path.splitext(path)[0] + ".json", "w") as f:
        json.dump(meta or {}, f, indent=1)


def load_weights(path: str) -> np.ndarray:
    w = np.load(path, allow_pickle=False)
    if w.dtype != np.float32 or w.shape != (10944,):
        raise ValueError("not a learned-stage checkpoint")
    return w


def validate(solver, net, rhs, rtol: float = 1e-10, max_it: int = 150, margin: float = 1e-3):
    """Plain and staged FGMRES on each right-hand side (float64 device tensors).
    The stage stays attached only if it cuts the iteration count on every one
    at the same tolerance; otherwise it is detached. Returns (enabled, rows)."""
    solver.attach_net(net, margin)
    rows = []
    for b in rhs:
        _, p = solver.fgmres_solve(b, rtol, max_it)
        _, q = solver.fgmres_solve(b, rtol, max_it, learned=True)
        rows.append({"plain": p["iterations"], "learned": q["iterations"], "plain_converged": p["converged"],
                     "learned_converged": q["converged"], "accepted": q["learned_accepted"],
                     "rejected": q["learned_rejected"]})
    enabled = bool(rows) and all(r["learned_converged"] and r["learned"] < r["plain"] for r in rows)
    if not enabled:
        solver.attach_net(None)
    return enabled, rows
