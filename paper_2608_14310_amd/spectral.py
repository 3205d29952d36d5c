"""Two-grid spectral diagnostic (Section 5.1, Table 1).

The iteration matrix T = I - B K_E of the solver's V-cycle is assembled on the
device column by column (`Solver.error_propagation` on unit vectors); its
eigenvalues are then computed on the host with the constant-pressure gauge
mode removed (T restricted to the velocity space times the mean-zero pressure
space, through an orthonormal basis of that space). With a two-level
hierarchy B is the two-grid operator the paper's Table 1 describes.
"""
from __future__ import annotations

from typing import Dict

import numpy as np


def iteration_matrix(solver, chunk: int = 512) -> np.ndarray:
    """Dense T = I - V K_E on the finest level (n x n, float64, host)."""
    import torch
    n = solver.n()
    T = np.empty((n, n))
    for k0 in range(0, n, chunk):
        k1 = min(n, k0 + chunk)
        X = torch.zeros((k1 - k0, n), dtype=torch.float64, device=solver.device)
        X[torch.arange(k1 - k0), torch.arange(k0, k1)] = 1.0
        T[:, k0:k1] = solver.error_propagation(X).cpu().numpy().T
    return T


def gauge_free_basis(N: int) -> np.ndarray:
    """Orthonormal basis (3N^2 x 3N^2-1) of velocities x mean-zero pressures."""
    n2 = N * N
    D = np.zeros((n2, n2 - 1))
    D[np.arange(n2 - 1), np.arange(n2 - 1)] = 1.0
    D[np.arange(1, n2), np.arange(n2 - 1)] = -1.0
    Qp, _ = np.linalg.qr(D)
    Q = np.zeros((3 * n2, 3 * n2 - 1))
    Q[:2 * n2, :2 * n2] = np.eye(2 * n2)
    Q[2 * n2:, 2 * n2:] = Qp
    return Q


def spectrum(T: np.ndarray, N: int) -> Dict[str, float]:
    """rho(T) and the extreme moduli of the preconditioned eigenvalues 1 - lambda(T)."""
    Q = gauge_free_basis(N)
    lam = np.linalg.eigvals(Q.T @ T @ Q)
    mod = np.abs(1.0 - lam)
    return {"rho_T": float(np.abs(lam).max()), "min_abs_lambda": float(mod.min()),
            "max_abs_lambda": float(mod.max())}
