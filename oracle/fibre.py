"""Flexible-fibre energies, force and tangent (Section 5.3) — test infrastructure.

The clamped flexible fibre of Section 5.3 is modelled by four discrete
energies of the marker positions X (M markers, component-interleaved vector
x[2k + c]) with links D_k = X_{k+1} - X_k (no periodic wrap: the fibre lies
inside the cell):

  bending     E_b = EI / (2 ds^5) * sum_{k=0}^{M-3} (D_k x D_{k+1})^2
  stretching  E_s = K_s / (2 ds)  * sum_{k=0}^{M-2} (|D_k| - ds)^2
  position    E_p = K_p / 2 * |X_m - X_c|^2
  tangent     E_t = K_t / 2 * |(X_{m+1} - X_{m-1}) / (2 ds) - e_x|^2

(a x b the scalar cross product, m the clamped midpoint marker). The force
density is F = -(1/ds) grad(E_b + E_s + E_p + E_t) and the Lagrangian E of
the linearised system is its tangent E = DF = -(1/ds) Hess(energy), which
couples the x and y components. Gradients and Hessians below are written
out term by term from those definitions; the tests pin them to finite
differences, invariances and closed forms.

Every function takes the links D as an optional argument. Section 5.3 updates
displacements and links incrementally, D^{n+1}_k = D^n_k + (the increment of
X_{k+1} - X_k), because on a nearly straight fibre the cross products of the
bending term sit far below the rounding of the absolute positions; a caller
that forms D that way passes it, and the tangent penalty uses
X_{m+1} - X_{m-1} = D_{m-1} + D_m so that it too sees the links.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _links(x, D=None):
    """Positions (M, 2) and links (M-1, 2): the given links D, else X_{k+1} - X_k."""
    X = np.asarray(x, dtype=np.float64).reshape(-1, 2)
    if D is None:
        return X, X[1:] - X[:-1]
    return X, np.asarray(D, dtype=np.float64).reshape(-1, 2)


def _cross(a, b):
    return a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]


def energy(x, p, D=None) -> float:
    """Total energy E_b + E_s + E_p + E_t at the interleaved positions x.
    p: dict with ds, EI, K_s, K_p, K_t, m (midpoint marker), Xc (2,).
    D: the links when the caller carries them (else differences of x)."""
    X, D = _links(x, D)
    ds = p["ds"]
    c = _cross(D[:-1], D[1:])
    Eb = p["EI"] / (2.0 * ds ** 5) * np.sum(c ** 2)
    L = np.linalg.norm(D, axis=1)
    Es = p["K_s"] / (2.0 * ds) * np.sum((L - ds) ** 2)
    m = p["m"]
    Ep = 0.5 * p["K_p"] * np.sum((X[m] - np.asarray(p["Xc"])) ** 2)
    g = (D[m - 1] + D[m]) / (2.0 * ds) - np.array([1.0, 0.0])   # X_{m+1} - X_{m-1}
    Et = 0.5 * p["K_t"] * np.sum(g ** 2)
    return float(Eb + Es + Ep + Et)


def gradient(x, p, parts=("b", "s", "p", "t"), D=None) -> np.ndarray:
    """d energy / dx (interleaved), summed over the named energies."""
    X, D = _links(x, D)
    M = len(X)
    ds = p["ds"]
    G = np.zeros((M, 2))
    if "b" in parts and M >= 3:
        a, b = D[:-1], D[1:]
        c = _cross(a, b)
        w = p["EI"] / ds ** 5 * c                      # d(EI/(2ds^5) c^2)/dc
        dca = np.stack([b[:, 1], -b[:, 0]], axis=1)     # dc/da
        dcb = np.stack([-a[:, 1], a[:, 0]], axis=1)     # dc/db
        # a = X_{k+1} - X_k, b = X_{k+2} - X_{k+1}
        np.add.at(G, np.arange(M - 2), -w[:, None] * dca)
        np.add.at(G, np.arange(1, M - 1), w[:, None] * (dca - dcb))
        np.add.at(G, np.arange(2, M), w[:, None] * dcb)
    if "s" in parts and M >= 2:
        L = np.linalg.norm(D, axis=1)
        gD = (p["K_s"] / ds * (L - ds) / L)[:, None] * D  # d E_s / d D_k
        np.add.at(G, np.arange(M - 1), -gD)
        np.add.at(G, np.arange(1, M), gD)
    m = p["m"]
    if "p" in parts:
        G[m] += p["K_p"] * (X[m] - np.asarray(p["Xc"]))
    if "t" in parts:
        g = (D[m - 1] + D[m]) / (2.0 * ds) - np.array([1.0, 0.0])
        G[m + 1] += p["K_t"] * g / (2.0 * ds)
        G[m - 1] -= p["K_t"] * g / (2.0 * ds)
    return G.ravel()


def force(x, p, D=None) -> np.ndarray:
    """Lagrangian force density F = -(1/ds) grad(energy) (Section 5.3)."""
    return -gradient(x, p, D=D) / p["ds"]


def hessian(x, p, parts=("b", "s", "p", "t"), D=None) -> sp.csr_matrix:
    """d^2 energy / dx^2 (2M x 2M, interleaved), summed over the named energies."""
    X, D = _links(x, D)
    M = len(X)
    ds = p["ds"]
    H = np.zeros((2 * M, 2 * M))

    def add(i, j, B):
        H[2 * i:2 * i + 2, 2 * j:2 * j + 2] += B

    if "b" in parts:
        R = np.array([[0.0, 1.0], [-1.0, 0.0]])          # c = a^T R b
        for k in range(M - 2):
            a, b = D[k], D[k + 1]
            c = a[0] * b[1] - a[1] * b[0]
            dca = np.array([b[1], -b[0]])
            dcb = np.array([-a[1], a[0]])
            # dc/dX for the markers k, k+1, k+2 (six coordinates)
            gX = np.concatenate([-dca, dca - dcb, dcb])
            # Hess_X c = T^T [[0, R], [R^T, 0]] T with T = [[-I, I, 0], [0, -I, I]]
            I2 = np.eye(2)
            T = np.block([[-I2, I2, np.zeros((2, 2))], [np.zeros((2, 2)), -I2, I2]])
            Hc = T.T @ np.block([[np.zeros((2, 2)), R], [R.T, np.zeros((2, 2))]]) @ T
            Hk = p["EI"] / ds ** 5 * (np.outer(gX, gX) + c * Hc)
            for r in range(3):
                for s_ in range(3):
                    add(k + r, k + s_, Hk[2 * r:2 * r + 2, 2 * s_:2 * s_ + 2])
    if "s" in parts:
        for k in range(M - 1):
            d = D[k]
            L = np.linalg.norm(d)
            A = p["K_s"] / ds * (np.eye(2) - (ds / L) * (np.eye(2) - np.outer(d, d) / L ** 2))
            add(k, k, A)
            add(k + 1, k + 1, A)
            add(k, k + 1, -A)
            add(k + 1, k, -A)
    m = p["m"]
    if "p" in parts:
        add(m, m, p["K_p"] * np.eye(2))
    if "t" in parts:
        B = p["K_t"] / (4.0 * ds ** 2) * np.eye(2)
        add(m + 1, m + 1, B)
        add(m - 1, m - 1, B)
        add(m + 1, m - 1, -B)
        add(m - 1, m + 1, -B)
    return sp.csr_matrix(H)


def tangent(x, p, D=None) -> sp.csr_matrix:
    """The Lagrangian E of the linearised system: E = DF = -(1/ds) Hess(energy),
    component-interleaved, coupling x and y (Section 5.3). Structure (a
    reading, the couplings the energies create): full 2 x 2 blocks for every
    pair of markers at most two apart along the fibre, stored even where a
    value is zero, so that the pattern does not depend on the configuration."""
    H = hessian(x, p, D=D).toarray()
    M = H.shape[0] // 2
    rows, cols = [], []
    for i in range(M):
        for j in range(max(0, i - 2), min(M, i + 3)):
            for a in range(2):
                for b in range(2):
                    rows.append(2 * i + a)
                    cols.append(2 * j + b)
    rows, cols = np.array(rows), np.array(cols)
    vals = -H[rows, cols] / p["ds"]
    return sp.csr_matrix((vals, (rows, cols)), shape=H.shape)
