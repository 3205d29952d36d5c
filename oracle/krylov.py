"""Right-preconditioned flexible GMRES (Section 5: zero initial guess,
Euclidean norm, stop at ||r_k||/||r_0|| <= rtol, no restarts).

The paper names FGMRES without details; this follows Saad's flexible GMRES:
z_j = B(v_j), w = K z_j, orthogonalise w against v_1..v_j, h_{j+1,j} = ||w||,
Givens rotations on the Hessenberg column, stop on the rotated residual
estimate |g_{j+1}| <= rtol * beta (or an exact breakdown h_{j+1,j} = 0), then
x = Z_k y with H_k y = g. Reading: classical Gram-Schmidt applied twice (CGS2);
`orth="mgs"` gives modified Gram-Schmidt as a cross-check.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List

import numpy as np


@dataclasses.dataclass
class FGMRESResult:
    x: np.ndarray
    iterations: int
    converged: bool
    history: List[float]          # relative residual estimate after each iteration
    breakdown: bool = False


def givens(a: float, b: float):
    """(c, s) with [c s; -s c] [a; b] = [hypot(a,b); 0]."""
    r = np.hypot(a, b)
    if r == 0.0:
        return 1.0, 0.0, 0.0
    return a / r, b / r, r


def fgmres(K: Callable[[np.ndarray], np.ndarray], B: Callable[[np.ndarray], np.ndarray], b: np.ndarray,
           rtol: float = 1e-10, max_it: int = 150, orth: str = "cgs2") -> FGMRESResult:
    n = b.shape[0]
    beta = float(np.linalg.norm(b))
    if beta == 0.0:
        return FGMRESResult(np.zeros(n), 0, True, [0.0])
    V = [b / beta]
    Z = []
    H = np.zeros((max_it + 1, max_it))
    cs, sn = np.zeros(max_it), np.zeros(max_it)
    g = np.zeros(max_it + 1)
    g[0] = beta
    hist = []
    k = 0
    converged = False
    breakdown = False
    for j in range(max_it):
        z = B(V[j])
        Z.append(z)
        w = K(z)
        if orth == "cgs2":
            Vm = np.stack(V, axis=1)
            h1 = Vm.T @ w
            w = w - Vm @ h1
            h2 = Vm.T @ w
            w = w - Vm @ h2
            H[:j + 1, j] = h1 + h2
        else:
            for i in range(j + 1):
                hij = float(V[i] @ w)
                H[i, j] = hij
                w = w - hij * V[i]
        hn = float(np.linalg.norm(w))
        H[j + 1, j] = hn
        # apply the stored rotations, then a new one
        for i in range(j):
            a, c = H[i, j], H[i + 1, j]
            H[i, j] = cs[i] * a + sn[i] * c
            H[i + 1, j] = -sn[i] * a + cs[i] * c
        c, s, r = givens(H[j, j], H[j + 1, j])
        cs[j], sn[j] = c, s
        H[j, j] = r
        H[j + 1, j] = 0.0
        g[j + 1] = -s * g[j]
        g[j] = c * g[j]
        k = j + 1
        rel = abs(g[j + 1]) / beta
        hist.append(rel)
        if rel <= rtol:
            converged = True
            break
        if hn == 0.0:
            converged = True
            breakdown = True
            break
        V.append(w / hn)
    y = np.zeros(k)
    for i in range(k - 1, -1, -1):
        y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
    x = np.stack(Z[:k], axis=1) @ y
    return FGMRESResult(x, k, converged, hist, breakdown)
