"""Study (oracle only, CPU): FGMRES with the multiplicative CAV V(1,1) cycle on
the open-fibre beam law at high bending stiffness, where the GPU solve was
seen to stall.

Test infrastructure like the rest of `oracle/`. For one beam system it
reports, per smoothed level, the largest 1-norm condition number of the
equilibrated patch matrices (Section 3.3), then runs right-preconditioned
FGMRES (Section 5) with the V(1,1) cycle (Section 4) and prints the residual
estimate after every iteration. Variants:

  order    explicit_first | standard_first   the two coloured orders
           lexicographic                      the paper's sequential order (Section 3.3)
  solve    lu        equilibrated LU solves (the oracle's local solve)
           explicit  the explicit inverse C K~^{-1} R formed once and applied as a
                     matrix-vector product (what the device smoother stores)

Usage: python -m oracle.study_stall N kappa_b order solve [max_it]
Output: one line per iteration, then a JSON summary line.
"""
from __future__ import annotations

import json
import sys
import time

import numpy as np
import scipy.linalg as sla

sys.path.insert(0, __file__.rsplit("/oracle/", 1)[0])

import workloads  # noqa: E402
from oracle import krylov, multigrid, smoothers  # noqa: E402


class ExplicitInverseSolvers(smoothers.PatchSolvers):
    """Local solves as explicit inverses M = C K~^{-1} R applied to R_p r."""

    def __init__(self, K, patches, standard, inject=None):
        super().__init__(K, patches, standard, inject)
        self.minv = []
        for (lu, rs, cs) in self.large_f:
            n = lu[0].shape[0]
            Ki = sla.lu_solve(lu, np.eye(n))
            self.minv.append(cs[:, None] * Ki * rs[None, :])

    def _large_solve(self, t, rp):
        return self.minv[t] @ rp


def level_conditions(H: multigrid.Hierarchy):
    """Largest kappa_1 of the equilibrated explicit-patch matrices per level."""
    out = []
    for l, lev in enumerate(H.levels):
        if lev.solvers is None:
            continue
        worst = 0.0
        for (lu, rs, cs), k in zip(lev.solvers.large_f, lev.solvers.large):
            Kt = smoothers.equilibrate(smoothers.dense_submatrix(lev.K, lev.patches[k]))[0]
            inv = sla.lu_solve(lu, np.eye(Kt.shape[0]))
            worst = max(worst, np.linalg.norm(Kt, 1) * np.linalg.norm(inv, 1))
        out.append(dict(level=l, N=lev.N, explicit=len(lev.solvers.large), max_cond1=worst))
    return out


def main(argv):
    N, kb, order, solve = int(argv[0]), float(argv[1]), argv[2], argv[3]
    max_it = int(argv[4]) if len(argv) > 4 else 150
    L = 5 if N == 512 else workloads.levels_to(N, 8)
    s = workloads.beam_fibres(N, L, kappa_b=kb, kappa_s=1e4, seed=0)
    t0 = time.time()
    if order == "lexicographic":
        H = multigrid.Hierarchy(s, alpha=1.0, smoother="multiplicative")
    else:
        H = multigrid.Hierarchy(s, alpha=1.0, smoother="coloured", order=order)
    if solve == "explicit":
        for lev in H.levels:
            if lev.solvers is not None:
                lev.solvers = ExplicitInverseSolvers(lev.K, lev.patches, lev.standard)
    conds = level_conditions(H)
    for c in conds:
        print("cond", json.dumps(c), flush=True)
    print(f"setup {time.time() - t0:.1f} s", flush=True)
    if order != "lexicographic" and solve == "explicit":
        # the coloured order builds its own solvers in patch order on first use
        for l, lev in enumerate(H.levels):
            if lev.solvers is None:
                continue
            H.smooth(l, np.zeros(lev.K.shape[0]), np.zeros(lev.K.shape[0]))
            lev.msolvers = ExplicitInverseSolvers(lev.K, lev.msolvers.patches, lev.standard[
                [c for ph in lev.phases for c in ph]])
    K = H.levels[-1].K
    count = [0]

    def prec(v):
        z = H.vcycle(v)
        count[0] += 1
        print(f"vcycle {count[0]} at {time.time() - t1:.1f} s", flush=True)
        return z

    def kop(z):
        return K @ z

    t1 = time.time()
    res = krylov.fgmres(kop, prec, s.b, 1e-10, max_it)
    for i, h in enumerate(res.history):
        print(f"it {i + 1} est {h:.6e}", flush=True)
    true = float(np.linalg.norm(s.b - K @ res.x) / np.linalg.norm(s.b))
    print(json.dumps(dict(N=N, kappa_b=kb, order=order, solve=solve, iterations=res.iterations,
                          converged=bool(res.converged), est=res.history[-1], true=true,
                          solve_s=round(time.time() - t1, 1), conds=conds)), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
