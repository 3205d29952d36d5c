"""Immersed-boundary coupling and force laws (Section 2, Section 5.2, Appendix A).

* phi4: Peskin's four-point kernel, the textbook closed form.
* J: velocity interpolation, U_k = sum_ij u_ij delta_h(x_face - X_k) h^2 with
  delta_h(x) = h^-2 phi(x/h) phi(y/h); so J_{k,face} = phi(.)phi(.) (Section 2).
* S = h^-2 J^T W, W = diag(omega) (Appendix A: S = (ds/h^2) J^T for omega = ds).
* E: Lagrangian elasticity, acting on each component separately for every
  linear law used here (springs Eq. disc_force_law; target points and closed
  beam Section 5.2; open fibres: second differences plus springs, a reading).
* E_E = S E J (Eq. intro_saddle).

Lagrangian ordering: component-interleaved, entry 2k + c for marker k,
component c (0 = x, 1 = y).

Kernel support (a reading): each marker touches the fixed 4 x 4 box of faces
with base index floor(X/h - sigma) - 1 per axis (sigma = face offset in cells),
and every face of that box is a structural entry of J even where phi is 0.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def phi4(r):
    """Peskin's 4-point kernel (Peskin 2002):
    (3 - 2|r| + sqrt(1 + 4|r| - 4 r^2))/8 for |r| <= 1,
    (5 - 2|r| - sqrt(-7 + 12|r| - 4 r^2))/8 for 1 <= |r| <= 2, 0 beyond."""
    a = np.abs(np.asarray(r, dtype=np.float64))
    out = np.zeros_like(a)
    m1 = a <= 1.0
    m2 = (a > 1.0) & (a <= 2.0)
    out[m1] = (3.0 - 2.0 * a[m1] + np.sqrt(np.maximum(1.0 + 4.0 * a[m1] - 4.0 * a[m1] ** 2, 0.0))) / 8.0
    out[m2] = (5.0 - 2.0 * a[m2] - np.sqrt(np.maximum(-7.0 + 12.0 * a[m2] - 4.0 * a[m2] ** 2, 0.0))) / 8.0
    return out


# face offsets in cell units: u at (i, j+1/2), v at (i+1/2, j)
_SIGMA = {0: (0.0, 0.5), 1: (0.5, 0.0)}


def interpolation(N: int, X: np.ndarray) -> sp.csr_matrix:
    """J: (2M) x (2N^2) with J[2k+c, face] = phi(i + sx - x/h) phi(j + sy - y/h)."""
    h = 1.0 / N
    M = X.shape[0]
    rows, cols, vals = [], [], []
    for c in (0, 1):
        sx, sy = _SIGMA[c]
        gx = X[:, 0] / h - sx
        gy = X[:, 1] / h - sy
        i0 = np.floor(gx).astype(np.int64) - 1
        j0 = np.floor(gy).astype(np.int64) - 1
        for a in range(4):
            for b in range(4):
                i = i0 + a
                j = j0 + b
                w = phi4(i - gx) * phi4(j - gy)
                rows.append(2 * np.arange(M) + c)
                cols.append(c * N * N + (i % N) * N + (j % N))
                vals.append(w)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(2 * M, 2 * N * N))


def structural_interpolation(N: int, X: np.ndarray) -> sp.csr_matrix:
    """All-ones copy of J's fixed 4x4-box pattern (used for patch patterns)."""
    J = interpolation(N, X)
    return sp.csr_matrix((np.ones_like(J.data), J.indices, J.indptr), shape=J.shape)


def spreading(N: int, J: sp.spmatrix, omega: np.ndarray) -> sp.csr_matrix:
    """S = h^-2 J^T W with W = diag(omega) on both components (Section 2)."""
    h = 1.0 / N
    W = sp.diags(np.repeat(omega, 2))
    return (J.T @ W / h ** 2).tocsr()


# ------------------------------------------------------------ force laws ---

def _circ(M, stencil):
    """Circulant M x M with a centred stencil (entries summed if the stencil wraps)."""
    h = len(stencil) // 2
    rows, cols, vals = [], [], []
    for k in range(M):
        for o, c in enumerate(stencil):
            rows.append(k)
            cols.append((k + o - h) % M)
            vals.append(c)
    return sp.csr_matrix((vals, (rows, cols)), shape=(M, M))


def _diff1_open(M):
    """(M-1) x M forward difference."""
    return sp.diags([-np.ones(M - 1), np.ones(M - 1)], [0, 1], shape=(M - 1, M), format="csr")


def _diff2_open(M):
    """(M-2) x M second difference."""
    return sp.diags([np.ones(M - 2), -2 * np.ones(M - 2), np.ones(M - 2)], [0, 1, 2],
                    shape=(M - 2, M), format="csr")


def segment_elasticity(law: str, kappa: dict, M: int, closed: bool, ds: float) -> sp.csr_matrix:
    """Scalar (per-component) elasticity matrix of one segment."""
    if law == "target":
        # E = -kappa_t I (Section 5.2)
        return (-kappa["kappa_t"] * sp.identity(M, format="csr")).tocsr()
    if law == "membrane":
        # F_k = kappa_s/ds^2 (X_{k+1} + X_{k-1} - 2 X_k) on a closed curve (Eq. disc_force_law)
        assert closed
        return (kappa["kappa_s"] / ds ** 2 * _circ(M, [1.0, -2.0, 1.0])).tocsr()
    if law == "beam_closed":
        # F = -kappa_b d^4X/ds^4, centred five-point stencil (Section 5.2)
        assert closed
        return (-kappa["kappa_b"] / ds ** 4 * _circ(M, [1.0, -4.0, 6.0, -4.0, 1.0])).tocsr()
    if law == "beam_open":
        # open fibre: bending via second differences plus stretching springs (a reading)
        assert not closed
        D2 = _diff2_open(M)
        D1 = _diff1_open(M)
        return (-kappa["kappa_b"] / ds ** 4 * (D2.T @ D2) - kappa["kappa_s"] / ds ** 2 * (D1.T @ D1)).tocsr()
    raise ValueError(law)


def elasticity(system) -> sp.csr_matrix:
    """Lagrangian E (2M x 2M, component-interleaved): each segment's scalar law
    on both components, no coupling between components or segments; for the
    flexible fibre (Section 5.3) the tangent of its nonlinear force, which
    couples the components (oracle.fibre)."""
    if system.law == "fibre":
        from . import fibre
        (seg,) = system.segments
        k = system.kappa
        p = dict(ds=seg.ds, EI=k["EI"], K_s=k["K_s"], K_p=k["K_p"], K_t=k["K_t"], m=int(k["m"]),
                 Xc=np.array([k["clamp_x"], k["clamp_y"]]))
        return fibre.tangent(np.asarray(seg.X, dtype=np.float64).ravel(), p)
    blocks = [segment_elasticity(system.law, system.kappa, len(s.X), s.closed, s.ds)
              for s in system.segments]
    Es = sp.block_diag(blocks, format="csr")
    return sp.kron(Es, sp.identity(2), format="csr")


def eulerian_elasticity(system):
    """E_E = S E J = h^-2 J^T W E J (Eq. intro_saddle).
    Returns (E_E, structural pattern as an all-ones matrix)."""
    N = system.N
    X = system.markers()
    omega = system.weights()
    J = interpolation(N, X)
    S = spreading(N, J, omega)
    E = elasticity(system)
    EE = (S @ E @ J).tocsr()
    # structural pattern: products of all-ones copies so no cancellation drops an entry
    Jo = structural_interpolation(N, X)
    Eo = sp.csr_matrix((np.ones_like(E.data), E.indices, E.indptr), shape=E.shape)
    pat = (Jo.T @ Eo @ Jo).tocsr()
    pat.data[:] = 1.0
    return EE, pat
