"""Reference solution of the reduced system (Eq. Eul_schur) by sparse LU.

The periodic K_E has the constant-pressure null mode (Section 5.1), so the
solution is taken in the mean-zero pressure space P_h^0 by solving the
bordered system [[K_E, e], [e^T, 0]] [x; lam] = [b; 0] with e the constant
pressure vector.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def bordered(K: sp.spmatrix, N: int) -> sp.csc_matrix:
    n = K.shape[0]
    e = np.zeros((n, 1))
    e[2 * N * N:, 0] = 1.0
    es = sp.csr_matrix(e)
    return sp.bmat([[K, es], [es.T, None]], format="csc")


def solve(K: sp.spmatrix, N: int, b: np.ndarray) -> np.ndarray:
    Bm = bordered(K, N)
    x = spla.splu(Bm).solve(np.concatenate([b, [0.0]]))
    return x[:-1]


def rounding_floor(K: sp.spmatrix, x: np.ndarray, b: np.ndarray) -> float:
    """u || |K| |x| ||_2 / ||b||_2 with u = 2^-53: the relative residual that
    rounding in one evaluation of b - K x can already produce."""
    Ka = abs(K)
    return float(2.0 ** -53 * np.linalg.norm(Ka @ np.abs(x)) / np.linalg.norm(b))
