"""Top-level oracle solve: hierarchy setup then FGMRES with one V-cycle per
iteration (Sections 4 and 5)."""
from __future__ import annotations

import time

import numpy as np

from . import direct, krylov, multigrid


def solve(system, alpha: float = 1.0, rtol: float = 1e-10, max_it: int = 150, family: str = "cav",
          smoother: str = "additive", orth: str = "cgs2", timings: dict = None):
    t0 = time.perf_counter()
    H = multigrid.Hierarchy(system, family=family, alpha=alpha, smoother=smoother)
    t1 = time.perf_counter()
    K = H.levels[-1].K
    res = krylov.fgmres(lambda x: K @ x, H.vcycle, system.b, rtol=rtol, max_it=max_it, orth=orth)
    t2 = time.perf_counter()
    if timings is not None:
        timings["setup"] = t1 - t0
        timings["solve"] = t2 - t1
    return H, res
