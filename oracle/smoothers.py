"""Patch relaxation (Section 3.3; Appendix A, Eq. additive_cav_saddle).

Local solves: K_p = R_p K_E R_p^T, built explicitly for every patch (no
sharing between patches). Before the LU factorisation each local matrix gets
one pass of max-norm row and then column equilibration (Section 3.3). Reading:
row scale r_i = 1/max_j |K_ij| and then column scale c_j = 1/max_i |r_i K_ij|,
each rounded to a power of two (2^(1-e) where the maximum is m 2^e, m in
[1/2, 1)) so the scaling is exact; the correction is delta = C K~^{-1} R r_p,
which equals K_p^{-1} r_p in exact arithmetic. LU with partial pivoting is
LAPACK's (scipy.linalg.lu_factor / numpy.linalg.solve).

Weighted additive sweep (Eq. additive_cav_saddle): from one residual
r = b - K_E w, every patch computes delta_p, and
w <- w + alpha sum_p R_p^T Theta_p delta_p with Theta_p = diag(1/cnt(d)),
the reciprocal-patch-count partition of unity named in Appendix A.
Multiplicative sweep (Section 3.3): patches in order, residual updated after
each correction. Both sweeps remove the mean pressure at the end (Section 3.3).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def pow2_recip(m):
    """2^(1-e) where m = f 2^e, f in [1/2,1); maps m into [1,2) exactly."""
    m = np.asarray(m, dtype=np.float64)
    _, e = np.frexp(m)
    return np.ldexp(1.0, 1 - e)


def equilibrate(Kp: np.ndarray):
    """Row then column max-norm scaling. Returns (Ktilde, rscale, cscale)."""
    rs = pow2_recip(np.max(np.abs(Kp), axis=-1))
    Kr = Kp * rs[..., :, None]
    cs = pow2_recip(np.max(np.abs(Kr), axis=-2))
    return Kr * cs[..., None, :], rs, cs


def dense_submatrix(K: sp.csr_matrix, idx: np.ndarray) -> np.ndarray:
    return K[idx][:, idx].toarray()


class PatchSolvers:
    """Factors for one level's patch family."""

    def __init__(self, K: sp.csr_matrix, patches, standard: np.ndarray, inject=None):
        self.K = K
        self.patches = patches
        self.n = K.shape[0]
        is5 = np.array([len(p) == 5 for p in patches])
        # stack the 5-unknown patches (solved as a batch of independent 5x5 systems)
        self.small = np.nonzero(is5)[0]
        self.large = np.nonzero(~is5)[0]
        self.inject = inject
        if len(self.small):
            idx = np.stack([patches[k] for k in self.small])                  # (ns, 5)
            rows = np.repeat(idx, 5, axis=1).ravel()
            cols = np.tile(idx, (1, 5)).ravel()
            Kp = np.asarray(K[rows, cols]).reshape(len(self.small), 5, 5)
            self.small_idx = idx
            self.small_Kt, self.small_rs, self.small_cs = equilibrate(Kp)
        self._pos = {}
        self.large_f = []
        for k in self.large:
            Kp = dense_submatrix(K, patches[k])
            Kt, rs, cs = equilibrate(Kp)
            self.large_f.append((sla.lu_factor(Kt, check_finite=True), rs, cs))

    def corrections(self, r: np.ndarray):
        """delta_p = K_p^{-1} R_p r for every patch, all from the same r.
        r may hold several right-hand sides as columns. Returns a list of
        arrays aligned with self.patches."""
        out = [None] * len(self.patches)
        extra = (1,) * (r.ndim - 1)
        if len(self.small):
            rs = self.small_rs.reshape(self.small_rs.shape + extra)
            cs = self.small_cs.reshape(self.small_cs.shape + extra)
            rhs = r[self.small_idx] * rs
            if r.ndim == 1:
                y = np.linalg.solve(self.small_Kt, rhs[..., None])[..., 0]
            else:
                y = np.linalg.solve(self.small_Kt, rhs)
            d = y * cs
            for t, k in enumerate(self.small):
                out[k] = d[t]
        for t, k in enumerate(self.large):
            out[k] = self._large_solve(t, r[self.patches[k]])
        return out

    def _large_solve(self, t, rp):
        lu, rs, cs = self.large_f[t]
        extra = (1,) * (rp.ndim - 1)
        return cs.reshape(cs.shape + extra) * sla.lu_solve(lu, rs.reshape(rs.shape + extra) * rp)

    def solve_one(self, k: int, rp: np.ndarray) -> np.ndarray:
        """delta = K_p^{-1} rp for patch k, using its stored equilibrated factors."""
        pos = self._pos.get(k)
        if pos is None:
            self._pos = {int(kk): ("s", t) for t, kk in enumerate(self.small)}
            self._pos.update({int(kk): ("l", t) for t, kk in enumerate(self.large)})
            pos = self._pos[k]
        kind, t = pos
        if kind == "s":
            extra = (1,) * (rp.ndim - 1)
            rs = self.small_rs[t].reshape((5,) + extra)
            cs = self.small_cs[t].reshape((5,) + extra)
            return cs * np.linalg.solve(self.small_Kt[t], rs * rp)
        return self._large_solve(t, rp)


def remove_mean_pressure(w: np.ndarray, N: int) -> np.ndarray:
    w = w.copy()
    p = w[2 * N * N:]
    p -= p.mean(axis=0)
    return w


def additive_sweep(K, solvers: PatchSolvers, cnt: np.ndarray, b, w, alpha: float, N: int):
    """One weighted additive sweep (Eq. additive_cav_saddle), then mean-pressure removal."""
    r = b - K @ w
    deltas = solvers.corrections(r)
    z = np.zeros_like(w)
    theta = 1.0 / cnt
    idx = np.concatenate(solvers.patches)
    th = theta[idx].reshape((len(idx),) + (1,) * (w.ndim - 1))
    np.add.at(z, idx, th * np.concatenate(deltas, axis=0))
    return remove_mean_pressure(w + alpha * z, N)


def seed_weights(N: int, patches) -> list:
    """Restricted-injection Theta for one-patch-per-cell families (Appendix A
    names restricted additive injection as the alternative to 1/cnt). Reading:
    the patch of cell (i,j) injects only into the standard Vanka unknowns of
    its own cell, V_ij, with weight 1 on p_ij and 1/2 on the four faces (each
    face belongs to the Vanka patches of its two incident cells), so that
    sum_i R_i^T Theta_i R_i = I."""
    n2 = N * N
    out = []
    for c, p in enumerate(patches):
        i, j = divmod(c, N)
        own = {i * N + j: 0.5, ((i + 1) % N) * N + j: 0.5, n2 + i * N + j: 0.5, n2 + i * N + (j + 1) % N: 0.5,
               2 * n2 + c: 1.0}
        out.append(np.array([own.get(int(d), 0.0) for d in p]))
    return out


def seed_restricted_sweep(K, solvers: PatchSolvers, theta, b, w, alpha: float, N: int):
    """Additive sweep of Eq. additive_cav_saddle with the restricted-injection
    Theta of `seed_weights`, then mean-pressure removal."""
    r = b - K @ w
    deltas = solvers.corrections(r)
    z = np.zeros_like(w)
    idx = np.concatenate(solvers.patches)
    th = np.concatenate(theta).reshape((len(idx),) + (1,) * (w.ndim - 1))
    np.add.at(z, idx, th * np.concatenate(deltas, axis=0))
    return remove_mean_pressure(w + alpha * z, N)


def restricted_additive_sweep(K, solvers: PatchSolvers, b, w, alpha: float, N: int):
    """Additive sweep with restricted injection (Appendix A's alternative
    choice of Theta): each patch writes only its injection mask."""
    r = b - K @ w
    deltas = solvers.corrections(r)
    z = np.zeros_like(w)
    for p, d, m in zip(solvers.patches, deltas, solvers.inject):
        z[p[m]] += d[m]
    return remove_mean_pressure(w + alpha * z, N)


def _update_columns(K, solvers: PatchSolvers, inject):
    """For each patch, the rows touched by K[:, q] (q the unknowns the patch
    updates: all of it, or its injected part) and K[rows, q] (CSC, the same
    columns in the same order), sliced once and kept on the solvers object
    for later sweeps with the same K. K[rows, q] @ d gives every touched row
    the sum K[:, q] @ d gives it, in the same order; the other rows are zero."""
    key = (id(K), inject is not None)
    cached = getattr(solvers, "_update_cols", None)
    if cached is None or cached[0] != key:
        Kc = K.tocsc()
        cols = []
        for k, p in enumerate(solvers.patches):
            q = p[inject[k]] if inject is not None else p
            Kq = Kc[:, q]
            rows = np.unique(Kq.indices)
            cols.append((rows, Kq[rows, :].tocsc()))
        cached = (key, cols)
        solvers._update_cols = cached
    return cached[1]


def multiplicative_sweep(K, solvers: PatchSolvers, b, w, N: int, inject=None):
    """Multiplicative Schwarz in the given patch order (Section 3.3). With
    `inject` masks only the unknowns of the unexpanded block are updated
    (restricted injection for box patches)."""
    cols = _update_columns(K, solvers, inject)
    w = w.copy()
    r = b - K @ w
    for k, p in enumerate(solvers.patches):
        d = solvers.solve_one(k, r[p])
        if inject is not None:
            m = inject[k]
            p, d = p[m], d[m]
        w[p] += d
        rows, Kq = cols[k]
        r[rows] -= Kq @ d
    return remove_mean_pressure(w, N)
