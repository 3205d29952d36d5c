"""Study (oracle only, CPU): which readings of the paper reproduce the two-grid
spectra of Table 1 (Section 5.1, N = 16 membrane, 8^2 coarse grid) and
Fig. 2 (N = 32, 16^2 coarse grid, B(1,0), B(4,2) and CAV).

Test infrastructure like the rest of `oracle/`. The two-grid operator is the
paper's B^TG: one multiplicative pre-sweep, an exact coarse solve, one
multiplicative post-sweep (Sections 3.3 and 4); T = I - B^TG K_E with the
constant-pressure mode removed, rho(T) its spectral radius, and the modulus
range of the nonzero eigenvalues of B^TG K_E (Section 5.1).

Readings varied (each is something the paper leaves open):
  placement  how the membrane's markers sit on the ellipse at spacing ~h/2:
             arclength (equal arclength, M = round(P/(h/2)); the default),
             ceil / floor (M rounded the other ways), shift (the same points
             moved half a spacing along the curve), angle (equal steps of
             the ellipse parameter), spacing_h (spacing ~h instead of h/2)
  order      the patch order of the multiplicative sweep: lex_i (cells
             (i, j) with i slowest; the default), lex_j (j slowest),
             explicit_first / standard_first (the two coloured orders)
  pattern    structural (E_E's fixed 4x4 kernel boxes; the default) or
             numerical (only the nonzero entries of the assembled E_E)

Usage: python -m oracle.study_table1 table1 | fig2
Output: one JSON line per case.
"""
from __future__ import annotations

import json
import math
import sys
import time

import numpy as np
import scipy.sparse as sp

sys.path.insert(0, __file__.rsplit("/oracle/", 1)[0])

import workloads  # noqa: E402
from oracle import ib, mac, multigrid, patches as pmod, smoothers  # noqa: E402

KAPPAS = (1e2, 1e3, 1e4, 1e5, 1e6)
PAPER_T1 = {1e2: (0.0816, 0.9357, 1.0486), 1e3: (0.1233, 0.9471, 1.1233), 1e4: (0.3518, 0.8470, 1.3518),
            1e5: (0.4684, 0.8090, 1.4684), 1e6: (0.5916, 0.8326, 1.5916)}


def ellipse_markers(N: int, placement: str) -> workloads.Segment:
    """The paper's membrane ellipse (centre (1/2, 1/2), semi-axes 0.23, 0.27)."""
    h = 1.0 / N
    ax, ay = 0.23, 0.27
    spacing = h if placement == "spacing_h" else h / 2
    t = np.linspace(0.0, 2.0 * math.pi, (1 << 18) + 1)
    x, y = 0.5 + ax * np.cos(t), 0.5 + ay * np.sin(t)
    s = np.concatenate([[0.0], np.cumsum(np.hypot(np.diff(x), np.diff(y)))])
    P = float(s[-1])
    M = {"ceil": math.ceil(P / spacing), "floor": math.floor(P / spacing)}.get(placement, int(round(P / spacing)))
    ds = P / M
    if placement == "angle":
        tk = 2.0 * math.pi * np.arange(M) / M
    else:
        off = 0.5 * ds if placement == "shift" else 0.0
        tk = np.interp(np.arange(M) * ds + off, s, t)
    X = np.stack([0.5 + ax * np.cos(tk), 0.5 + ay * np.sin(tk)], axis=1)
    return workloads.Segment(np.mod(X, 1.0), True, ds)


def membrane(N: int, kappa: float, mu: float, placement: str) -> workloads.System:
    h = 1.0 / N
    return workloads.System(f"study_membrane_N{N}_{placement}", N, 2, 1.0, mu, h / 2, "membrane",
                            {"kappa_s": kappa}, [ellipse_markers(N, placement)], np.zeros(3 * N * N))


def numerical_pattern(H: multigrid.Hierarchy):
    """Replace every level's patch pattern by the nonzeros of its assembled E_E."""
    for lev in H.levels:
        P = lev.EE.tocsr().copy()
        P.eliminate_zeros()
        P.data[:] = 1.0
        lev.pattern = P


def two_grid(system, family: str, order: str, pattern: str = "structural", box=(4, 2)):
    H = multigrid.Hierarchy(system, family=family, smoother="multiplicative", box=box)
    lev = H.levels[1]
    N = lev.N
    if pattern == "numerical" and family == "cav":
        numerical_pattern(H)
        lev.patches, lev.standard = pmod.cav_patches(N, lev.pattern)
    ncell = len(lev.patches)
    if family == "box":
        nb = N // box[0]
        blocks = [(I, J) for I in range(nb) for J in range(nb)]
        idx = list(range(ncell)) if order == "lex_i" else sorted(range(ncell), key=lambda k: (blocks[k][1], blocks[k][0]))
        inject = [lev.inject[k] for k in idx]
    else:
        inject = None
        if order == "lex_i":
            idx = list(range(ncell))
        elif order == "lex_j":
            idx = sorted(range(ncell), key=lambda c: (c % N, c // N))
        else:
            stencil = mac.reduced_operator(N, 1.0, 1.0, 1.0, sp.csr_matrix((2 * N * N, 2 * N * N)))
            phases = pmod.coloured_order(N, lev.patches, lev.pattern, stencil,
                                         standard_first=order == "standard_first")
            idx = [c for ph in phases for c in ph]
    sol = smoothers.PatchSolvers(lev.K, [lev.patches[k] for k in idx], np.asarray(lev.standard)[idx], inject)
    R, P = H.transfers(1)
    K = lev.K

    def smooth(b, w):
        return smoothers.multiplicative_sweep(K, sol, b, w, N, inject)

    n = K.shape[0]
    Bm = np.eye(n)
    x = smooth(Bm, np.zeros_like(Bm))
    x = x + P @ H.coarse_solve(R @ (Bm - K @ x))
    Bm = smooth(Bm, x)
    T = np.eye(n) - Bm @ K.toarray()
    # gauge: restrict to mean-free pressures
    D = np.zeros((N * N, N * N - 1))
    D[np.arange(N * N - 1), np.arange(N * N - 1)] = 1
    D[np.arange(1, N * N), np.arange(N * N - 1)] = -1
    Qp, _ = np.linalg.qr(D)
    Q = np.zeros((n, n - 1))
    Q[:2 * N * N, :2 * N * N] = np.eye(2 * N * N)
    Q[2 * N * N:, 2 * N * N:] = Qp
    lam = np.linalg.eigvals(Q.T @ T @ Q)
    mod = np.abs(1 - lam)
    return float(np.abs(lam).max()), float(mod.min()), float(mod.max())


def table1():
    for placement in ("arclength", "ceil", "floor", "shift", "angle", "spacing_h"):
        for order in ("lex_i", "lex_j", "explicit_first", "standard_first"):
            if placement != "arclength" and order not in ("lex_i", "lex_j"):
                continue
            for pattern in ("structural", "numerical"):
                if pattern == "numerical" and (placement != "arclength" or order != "lex_i"):
                    continue
                for k in KAPPAS:
                    t0 = time.time()
                    s = membrane(16, k, 1e-2, placement)
                    rho, lo, hi = two_grid(s, "cav", order, pattern)
                    print(json.dumps(dict(study="table1", placement=placement, order=order, pattern=pattern,
                                          kappa_s=k, M=s.M, rho_T=round(rho, 4), min_abs=round(lo, 4),
                                          max_abs=round(hi, 4), paper=PAPER_T1[k],
                                          seconds=round(time.time() - t0, 1))), flush=True)


def fig2():
    cases = [("vanka", (1, 0), 1.0, 0.88), ("box", (4, 2), 1.0, 0.13), ("box", (4, 2), 1e-2, 0.81),
             ("cav", None, 1e-2, 0.14)]
    for placement in ("arclength", "angle"):
        for family, box, mu, paper in cases:
            for order in ("lex_i", "lex_j"):
                t0 = time.time()
                s = membrane(32, 1e4, mu, placement)
                rho, lo, hi = two_grid(s, family, order, box=box or (4, 2))
                label = "CAV" if family == "cav" else f"B({box[0]},{box[1]})"
                print(json.dumps(dict(study="fig2", placement=placement, patches=label, mu=mu, order=order,
                                      rho_T=round(rho, 4), paper_rho_T=paper, seconds=round(time.time() - t0, 1))),
                      flush=True)


if __name__ == "__main__":
    {"table1": table1, "fig2": fig2}[sys.argv[1]]()
