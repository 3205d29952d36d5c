"""Grid transfers and Galerkin coarse elasticity (Section 4).

Velocity prolongation: lowest-order Raviart-Thomas interpolation on the coarse
quadrilaterals. A coarse u face (I,J) covers fine faces (2I,2J) and (2I,2J+1)
(weight 1); the fine faces halfway between coarse faces, (2I+1, 2J) and
(2I+1, 2J+1), take the mean of coarse faces (I,J) and (I+1,J). v is the same
with the axes swapped. Velocity restriction R = P^* = (1/4) P^T.
Pressure: bilinear prolongation (weights 9/16, 3/16, 3/16, 1/16, periodic,
a reading of "bilinear interpolation" on the periodic grid) and restriction by
averaging the four child cells.
Coarse elasticity: E_E^(l-1) = R E_E^(l) P.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .mac import iu


def prolong_velocity(Nc: int) -> sp.csr_matrix:
    Nf = 2 * Nc
    I, J = np.meshgrid(np.arange(Nc), np.arange(Nc), indexing="ij")
    I, J = I.ravel(), J.ravel()
    rows, cols, vals = [], [], []

    def add(r, c, w):
        rows.append(r)
        cols.append(c)
        vals.append(np.full(r.shape, w))

    # u (x-faces)
    cu = iu(Nc, I, J)
    cu_right = iu(Nc, I + 1, J)
    for dj in (0, 1):
        add(iu(Nf, 2 * I, 2 * J + dj), cu, 1.0)
        add(iu(Nf, 2 * I + 1, 2 * J + dj), cu, 0.5)
        add(iu(Nf, 2 * I + 1, 2 * J + dj), cu_right, 0.5)
    # v (y-faces)
    cv = Nc * Nc + iu(Nc, I, J)
    cv_up = Nc * Nc + iu(Nc, I, J + 1)
    for di in (0, 1):
        add(Nf * Nf + iu(Nf, 2 * I + di, 2 * J), cv, 1.0)
        add(Nf * Nf + iu(Nf, 2 * I + di, 2 * J + 1), cv, 0.5)
        add(Nf * Nf + iu(Nf, 2 * I + di, 2 * J + 1), cv_up, 0.5)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(2 * Nf * Nf, 2 * Nc * Nc))


def restrict_velocity(Nc: int) -> sp.csr_matrix:
    """R = (1/4) P^T (Section 4)."""
    return (0.25 * prolong_velocity(Nc).T).tocsr()


def prolong_pressure(Nc: int) -> sp.csr_matrix:
    """Bilinear interpolation from coarse to fine cell centres, periodic.
    Fine cell (2I+a, 2J+b) lies a quarter coarse cell from the centre of coarse
    cell (I,J), towards neighbour (I + (2a-1), J + (2b-1))."""
    Nf = 2 * Nc
    I, J = np.meshgrid(np.arange(Nc), np.arange(Nc), indexing="ij")
    I, J = I.ravel(), J.ravel()
    rows, cols, vals = [], [], []
    for a in (0, 1):
        for b in (0, 1):
            r = iu(Nf, 2 * I + a, 2 * J + b)
            sx, sy = 2 * a - 1, 2 * b - 1
            for (di, dj, w) in ((0, 0, 9 / 16), (sx, 0, 3 / 16), (0, sy, 3 / 16), (sx, sy, 1 / 16)):
                rows.append(r)
                cols.append(iu(Nc, I + di, J + dj))
                vals.append(np.full(r.shape, w))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(Nf * Nf, Nc * Nc))


def restrict_pressure(Nc: int) -> sp.csr_matrix:
    """Cell averaging: coarse p(I,J) = mean of the four fine children."""
    Nf = 2 * Nc
    I, J = np.meshgrid(np.arange(Nc), np.arange(Nc), indexing="ij")
    I, J = I.ravel(), J.ravel()
    rows, cols = [], []
    for a in (0, 1):
        for b in (0, 1):
            rows.append(iu(Nc, I, J))
            cols.append(iu(Nf, 2 * I + a, 2 * J + b))
    rows = np.concatenate(rows)
    return sp.csr_matrix((np.full(rows.shape, 0.25), (rows, np.concatenate(cols))), shape=(Nc * Nc, Nf * Nf))


def prolongation(Nc: int) -> sp.csr_matrix:
    """Full [u;v;p] prolongation."""
    return sp.block_diag([prolong_velocity(Nc), prolong_pressure(Nc)], format="csr")


def restriction(Nc: int) -> sp.csr_matrix:
    """Full [u;v;p] restriction."""
    return sp.block_diag([restrict_velocity(Nc), restrict_pressure(Nc)], format="csr")


def galerkin(EEf: sp.spmatrix, pat_f: sp.spmatrix, Nc: int):
    """E_E^(l-1) = R E_E^(l) P and its structural pattern (Section 4)."""
    P = prolong_velocity(Nc)
    R = restrict_velocity(Nc)
    EEc = (R @ EEf @ P).tocsr()
    Po = sp.csr_matrix((np.ones_like(P.data), P.indices, P.indptr), shape=P.shape)
    patc = (Po.T @ pat_f @ Po).tocsr()
    patc.data[:] = 1.0
    return EEc, patc
