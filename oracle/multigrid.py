"""Geometric multigrid V(1,1) preconditioner (Section 4).

Levels are numbered 0 (coarsest) .. L-1 (finest), grids halving each time.
Every level rediscretises the Stokes part with its own h and uses the Galerkin
elasticity E_E^(l-1) = R E_E^(l) P. Every level except the coarsest gets the
chosen patch family and its local factors; the coarsest system is solved by a
precomputed direct factorisation. Reading: the periodic coarse operator has the
constant-pressure null mode (Section 5.1), so the coarse solve uses the
bordered matrix [[K_0, e], [e^T, 0]] with e the constant pressure vector.
Reading: pre-smoothing starts from zero; one pre- and one post-sweep (the
paper's V(1,1); `pre` and `post` repeat the sweeps, each from the iterate the
previous one left); the smoothers remove the mean pressure after every sweep.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import hierarchy, ib, mac, patches as pmod, smoothers


@dataclasses.dataclass
class Level:
    N: int
    K: sp.csr_matrix
    EE: sp.csr_matrix
    pattern: sp.csr_matrix
    patches: Optional[list] = None
    standard: Optional[np.ndarray] = None
    inject: Optional[list] = None
    cnt: Optional[np.ndarray] = None
    solvers: Optional[smoothers.PatchSolvers] = None
    theta: Optional[list] = None
    phases: Optional[list] = None
    msolvers: Optional[smoothers.PatchSolvers] = None
    minject: Optional[list] = None


class Hierarchy:
    def __init__(self, system, family: str = "cav", alpha: float = 1.0, smoother: str = "additive",
                 box=(4, 2), order: str = "standard_first", lex: str = "y_fast", pre: int = 1, post: int = 1):
        """lex: the reading of the paper's lexicographic patch order for the
        sequential multiplicative smoother (Section 3.3): "y_fast" visits
        cells (i, j) with the y index j fastest (the vector layout's order),
        "x_fast" with the x index i fastest (boxes by their lower-left cells
        alike). pre, post: smoothing sweeps before and after the coarse
        correction (V(pre, post))."""
        self.system = system
        self.pre = pre
        self.post = post
        self.order = order
        self.lex = lex
        self.alpha = alpha
        self.smoother = smoother
        self.family = family
        L = system.n_levels
        EE, pat = ib.eulerian_elasticity(system)
        ee = [None] * L
        ee[L - 1] = (EE, pat)
        for l in range(L - 1, 0, -1):
            Nc = system.N >> (L - l)
            ee[l - 1] = hierarchy.galerkin(ee[l][0], ee[l][1], Nc)
        self.levels: List[Level] = []
        for l in range(L):
            N = system.N >> (L - 1 - l)
            K = mac.reduced_operator(N, system.rho, system.mu, system.dt, ee[l][0])
            self.levels.append(Level(N, K, ee[l][0], ee[l][1]))
        for l in range(1, L):
            lev = self.levels[l]
            if family == "cav":
                lev.patches, lev.standard = pmod.cav_patches(lev.N, lev.pattern)
            elif family == "vanka":
                lev.patches, lev.standard = pmod.vanka_patches(lev.N)
            elif family == "box":
                lev.patches, lev.inject = pmod.box_patches(lev.N, *box)
                lev.standard = np.zeros(len(lev.patches), dtype=bool)
            else:
                raise ValueError(family)
            lev.cnt = pmod.patch_counts(lev.K.shape[0], lev.patches)
            if smoother == "multiplicative" and lex == "x_fast":
                # the same patches, visited with the x index fastest
                if family == "box":
                    nb = lev.N // box[0]
                    perm = sorted(range(len(lev.patches)), key=lambda k: (k % nb, k // nb))
                else:
                    perm = sorted(range(len(lev.patches)), key=lambda c: (c % lev.N, c // lev.N))
                lev.patches = [lev.patches[k] for k in perm]
                lev.standard = np.asarray(lev.standard)[perm]
                if lev.inject is not None:
                    lev.inject = [lev.inject[k] for k in perm]
            lev.solvers = smoothers.PatchSolvers(lev.K, lev.patches, lev.standard, lev.inject)
        # coarsest: dense bordered LU
        K0 = self.levels[0].K.toarray()
        n0 = K0.shape[0]
        N0 = self.levels[0].N
        B = np.zeros((n0 + 1, n0 + 1))
        B[:n0, :n0] = K0
        B[2 * N0 * N0:n0, n0] = 1.0
        B[n0, 2 * N0 * N0:n0] = 1.0
        self.coarse_lu = sla.lu_factor(B)

    def coarse_solve(self, b: np.ndarray) -> np.ndarray:
        n0 = b.shape[0]
        x = sla.lu_solve(self.coarse_lu, np.concatenate([b, np.zeros((1,) + b.shape[1:])], axis=0))
        return x[:n0]

    def smooth(self, l: int, b: np.ndarray, w: np.ndarray) -> np.ndarray:
        lev = self.levels[l]
        if self.smoother == "additive":
            if self.family == "box":
                return smoothers.restricted_additive_sweep(lev.K, lev.solvers, b, w, self.alpha, lev.N)
            return smoothers.additive_sweep(lev.K, lev.solvers, lev.cnt, b, w, self.alpha, lev.N)
        if self.smoother == "restricted":
            if lev.theta is None:
                lev.theta = smoothers.seed_weights(lev.N, lev.patches)
            return smoothers.seed_restricted_sweep(lev.K, lev.solvers, lev.theta, b, w, self.alpha, lev.N)
        if self.smoother == "multiplicative":
            return smoothers.multiplicative_sweep(lev.K, lev.solvers, b, w, lev.N, lev.inject)
        if self.smoother == "coloured" and self.family == "box":
            if lev.phases is None:
                stencil = mac.reduced_operator(lev.N, 1.0, 1.0, 1.0, sp.csr_matrix((2 * lev.N ** 2, 2 * lev.N ** 2)))
                lev.phases = pmod.coloured_box_order(lev.N, lev.patches, lev.pattern, stencil)
                order = [k for ph in lev.phases for k in ph]
                lev.minject = [lev.inject[k] for k in order]
                lev.msolvers = smoothers.PatchSolvers(lev.K, [lev.patches[k] for k in order], lev.standard[order],
                                                      lev.minject)
            return smoothers.multiplicative_sweep(lev.K, lev.msolvers, b, w, lev.N, lev.minject)
        if self.smoother == "coloured":
            if lev.phases is None:
                # structural stencil pattern (unit coefficients so no coupling vanishes when mu = 0)
                stencil = mac.reduced_operator(lev.N, 1.0, 1.0, 1.0, sp.csr_matrix((2 * lev.N ** 2, 2 * lev.N ** 2)))
                lev.phases = pmod.coloured_order(lev.N, lev.patches, lev.pattern, stencil,
                                                 standard_first=self.order == "standard_first")
                order = [c for ph in lev.phases for c in ph]
                lev.msolvers = smoothers.PatchSolvers(lev.K, [lev.patches[c] for c in order], lev.standard[order])
            return smoothers.multiplicative_sweep(lev.K, lev.msolvers, b, w, lev.N)
        raise ValueError(self.smoother)

    def vcycle(self, b: np.ndarray, l: Optional[int] = None) -> np.ndarray:
        """V(l, b): x = 0; x = S(b, x) pre times; x += P V(l-1, R(b - K x));
        x = S(b, x) post times."""
        if l is None:
            l = len(self.levels) - 1
        if l == 0:
            return self.coarse_solve(b)
        lev = self.levels[l]
        R, P = self.transfers(l)
        x = np.zeros_like(b)
        for _ in range(self.pre):
            x = self.smooth(l, b, x)
        r = b - lev.K @ x
        ec = self.vcycle(R @ r, l - 1)
        x = x + P @ ec
        for _ in range(self.post):
            x = self.smooth(l, b, x)
        return x

    def transfers(self, l: int):
        """(restriction to level l-1, prolongation from level l-1)."""
        if not hasattr(self, "_tr"):
            self._tr = {}
        if l not in self._tr:
            Nc = self.levels[l - 1].N
            self._tr[l] = (hierarchy.restriction(Nc), hierarchy.prolongation(Nc))
        return self._tr[l]

    def patch_stats(self):
        out = []
        for l, lev in enumerate(self.levels):
            if lev.patches is None:
                continue
            sizes = np.array([len(p) for p in lev.patches])
            out.append(dict(level=l, N=lev.N, count=len(sizes), enlarged=int((~lev.standard).sum()),
                            avg=float(sizes.mean()), max=int(sizes.max()),
                            sum_np2_enlarged=int((sizes[~lev.standard] ** 2).sum())))
        return out
