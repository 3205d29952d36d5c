"""Periodic MAC-grid operators (Section 2; Eq. intro_saddle and Eq. Eul_schur).

Unknown ordering (a reading; the paper fixes no global order): the vector is
[u ; v ; p], each block an N x N array indexed [i][j] with i the x index (slow)
and j the y index (fast). u_ij sits at (i h, (j+1/2) h), v_ij at
((i+1/2) h, j h), p_ij at the cell centre. Indices are periodic mod N.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def iu(N, i, j):
    return (np.asarray(i) % N) * N + (np.asarray(j) % N)


def iv(N, i, j):
    return N * N + iu(N, i, j)


def ip(N, i, j):
    return 2 * N * N + iu(N, i, j)


def _grid(N):
    i, j = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    return i.ravel(), j.ravel()


def divergence(N: int, h: float) -> sp.csr_matrix:
    """D: velocity -> cell centres, (Du)_ij = (u_{i+1,j} - u_ij + v_{i,j+1} - v_ij)/h.
    Columns index the velocity block only (2N^2)."""
    i, j = _grid(N)
    row = iu(N, i, j)
    rows = np.concatenate([row, row, row, row])
    cols = np.concatenate([iu(N, i + 1, j), iu(N, i, j), N * N + iu(N, i, j + 1), N * N + iu(N, i, j)])
    vals = np.concatenate([np.full(N * N, 1 / h), np.full(N * N, -1 / h),
                           np.full(N * N, 1 / h), np.full(N * N, -1 / h)])
    return sp.csr_matrix((vals, (rows, cols)), shape=(N * N, 2 * N * N))


def gradient(N: int, h: float) -> sp.csr_matrix:
    """G = -D^T (the standard MAC relation stated in Section 2)."""
    return (-divergence(N, h).T).tocsr()


def scalar_laplacian(N: int, h: float) -> sp.csr_matrix:
    """Periodic 5-point Laplacian on an N x N array indexed [i][j]."""
    i, j = _grid(N)
    row = iu(N, i, j)
    rows = np.concatenate([row] * 5)
    cols = np.concatenate([iu(N, i + 1, j), iu(N, i - 1, j), iu(N, i, j + 1), iu(N, i, j - 1), row])
    vals = np.concatenate([np.full(4 * N * N, 1 / h ** 2), np.full(N * N, -4 / h ** 2)])
    return sp.csr_matrix((vals, (rows, cols)), shape=(N * N, N * N))


def vector_laplacian(N: int, h: float) -> sp.csr_matrix:
    Ls = scalar_laplacian(N, h)
    return sp.block_diag([Ls, Ls], format="csr")


def momentum_A0(N: int, h: float, rho: float, mu: float, dt: float) -> sp.csr_matrix:
    """A0 = (rho/dt) I - mu L (Eq. intro_saddle)."""
    return (rho / dt * sp.identity(2 * N * N, format="csr") - mu * vector_laplacian(N, h)).tocsr()


def reduced_operator(N: int, rho: float, mu: float, dt: float, EE: sp.spmatrix) -> sp.csr_matrix:
    """K_E = [[A, G], [-D, 0]] with A = A0 - dt E_E (Eq. intro_saddle, Eq. Eul_schur)."""
    h = 1.0 / N
    A = momentum_A0(N, h, rho, mu, dt) - dt * EE
    D = divergence(N, h)
    G = gradient(N, h)
    return sp.bmat([[A, G], [-D, None]], format="csr")
