"""Patch families (Section 3.1 and Section 3.2, Eq. cav_patch_set).

Every patch is a sorted array of global unknown indices in the [u; v; p]
ordering of `oracle.mac`.

* Standard pressure-centred Vanka patch V_ij = {p_ij} U U_ij with
  U_ij = {u_ij, u_{i+1,j}, v_ij, v_{i,j+1}}.
* V(C) = union of V_c over a cell set C.
* CAV: U_hat = U_ij plus every velocity k with (E_E)_{kl} != 0 or
  (E_E)_{lk} != 0 for some l in U_ij; if U_hat = U_ij the patch is V_ij,
  otherwise V(C(U_hat)) with C(u_ij) = {(i-1,j),(i,j)}, C(v_ij) = {(i,j-1),(i,j)}.
  "Nonzero" is read structurally (a reading): the pattern is that of the
  all-ones products, so no numerical cancellation removes a coupling.
* Box B(b,o): b x b cell blocks expanded by o layers; restricted injection
  keeps only the unknowns of the unexpanded block (Section 3.3).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .mac import iu


def cell_velocities(N: int, i: int, j: int):
    """U_ij as global indices."""
    return [int(iu(N, i, j)), int(iu(N, i + 1, j)), N * N + int(iu(N, i, j)), N * N + int(iu(N, i, j + 1))]


def vanka_patch(N: int, i: int, j: int) -> np.ndarray:
    return np.array(sorted([2 * N * N + int(iu(N, i, j))] + cell_velocities(N, i, j)), dtype=np.int64)


def union_patch(N: int, cells) -> np.ndarray:
    """V(C) for a set of cells C."""
    s = set()
    for (a, b) in cells:
        s.add(2 * N * N + int(iu(N, a, b)))
        s.update(cell_velocities(N, a, b))
    return np.array(sorted(s), dtype=np.int64)


def incident_cells(N: int, dof: int):
    """C(w): the two cells whose divergence rows contain velocity w."""
    if dof < N * N:
        i, j = divmod(dof, N)
        return [((i - 1) % N, j), (i, j)]
    d = dof - N * N
    i, j = divmod(d, N)
    return [(i, (j - 1) % N), (i, j)]


def cav_patches(N: int, pattern: sp.spmatrix):
    """One CAV patch per cell, in lexicographic cell order (i first).

    Returns (patches, standard) where standard[c] is True when U_hat = U
    for cell c = i*N + j.
    """
    P = (pattern != 0).astype(np.int8)
    Ps = ((P + P.T) != 0).tocsr()
    row_nnz = np.diff(Ps.indptr)
    patches = []
    standard = np.zeros(N * N, dtype=bool)
    for i in range(N):
        for j in range(N):
            U = cell_velocities(N, i, j)
            if all(row_nnz[d] == 0 for d in U):
                patches.append(vanka_patch(N, i, j))
                standard[i * N + j] = True
                continue
            Uhat = set(U)
            for d in U:
                Uhat.update(Ps.indices[Ps.indptr[d]:Ps.indptr[d + 1]].tolist())
            if Uhat == set(U):
                patches.append(vanka_patch(N, i, j))
                standard[i * N + j] = True
                continue
            cells = set()
            for w in Uhat:
                cells.update(incident_cells(N, w))
            patches.append(union_patch(N, cells))
    return patches, standard


def vanka_patches(N: int):
    """B(1,0): the standard Vanka family."""
    return [vanka_patch(N, i, j) for i in range(N) for j in range(N)], np.ones(N * N, dtype=bool)


def box_patches(N: int, b: int, o: int):
    """B(b,o) patches and their restricted-injection masks (Section 3.1, 3.3).

    Block lower-left cells visited in lexicographic order; returns
    (patches, inject) where inject[k] is a boolean mask over patches[k] that
    keeps the unknowns of the unexpanded b x b block V(block)."""
    assert N % b == 0
    patches, inject = [], []
    for I in range(0, N, b):
        for J in range(0, N, b):
            ext = [((I + r) % N, (J + s) % N) for r in range(-o, b + o) for s in range(-o, b + o)]
            core = [((I + r) % N, (J + s) % N) for r in range(b) for s in range(b)]
            patch = union_patch(N, ext)
            core_dofs = set(union_patch(N, core).tolist())
            patches.append(patch)
            inject.append(np.array([d in core_dofs for d in patch.tolist()]))
    return patches, inject


def coloured_order(N: int, patches, ee_pattern, stencil_K, standard_first: bool = False) -> list:
    """A multiplicative ordering whose consecutive runs ("phases") hold
    mutually independent patches: no shared unknown and no structural K_E
    entry between them, so applying a phase simultaneously equals applying its
    patches one after another in any order.

    Reading (the paper visits patches lexicographically; this order is the
    parallel one): patches whose velocity rows carry E_E entries come first,
    greedily coloured in order of decreasing size (ties by cell index), each
    taking the smallest colour not used by a conflicting, already coloured
    patch; then the E_E-free standard patches in 8 phases by colour
    (i + 3 j) mod 8, which separates every pair of standard patches coupled
    by the MAC stencils (with standard_first, those 8 phases come first).
    Returns a list of phases, each a sorted list of cells.
    """
    n2 = N * N
    P = ee_pattern.tocsr()
    rows_ee = np.diff(P.indptr) > 0
    # stencil_K is only a pattern source: rebuild-free structural pattern of its entries
    Kb = (abs(stencil_K) + sp.identity(stencil_K.shape[0])).tocsr()
    Kb.data[:] = 1.0
    Kb = Kb + sp.bmat([[(P + P.T), None], [None, sp.csr_matrix((n2, n2))]])
    Kb = (Kb != 0).tocsr()
    expl = []
    for c in range(n2):
        i, j = divmod(c, N)
        if any(rows_ee[d] for d in cell_velocities(N, i, j)):
            expl.append(c)
    owners = {}
    for c in expl:
        for d in patches[c].tolist():
            owners.setdefault(d, []).append(c)
    colour = {}
    for c in sorted(expl, key=lambda c: (-len(patches[c]), c)):
        reach = np.unique(Kb[patches[c]].indices)
        used = set()
        for d in reach.tolist():
            for q in owners.get(d, ()):
                if q in colour:
                    used.add(colour[q])
        k = 0
        while k in used:
            k += 1
        colour[c] = k
    exp_phases = []
    if colour:
        for k in range(max(colour.values()) + 1):
            exp_phases.append(sorted(c for c in expl if colour[c] == k))
    ex = set(expl)
    rest = [c for c in range(n2) if c not in ex]
    std_phases = [[c for c in rest if ((c // N) + 3 * (c % N)) % 8 == k] for k in range(8)]
    phases = std_phases + exp_phases if standard_first else exp_phases + std_phases
    return [p for p in phases if p]


def coloured_box_order(N: int, patches, ee_pattern, stencil_K) -> list:
    """A multiplicative ordering of the B(b,o) box family (reading: the paper
    visits boxes in lexicographic order of their blocks; this is the parallel
    form): boxes greedily coloured in order of decreasing size, ties by block
    order, on the same conflict graph as `coloured_order` (a shared unknown or a
    structural K_E entry between two boxes). Returns phases of box indices."""
    n2 = N * N
    P = ee_pattern.tocsr()
    Kb = (abs(stencil_K) + sp.identity(stencil_K.shape[0])).tocsr()
    Kb.data[:] = 1.0
    Kb = (Kb + sp.bmat([[(P + P.T), None], [None, sp.csr_matrix((n2, n2))]]) != 0).tocsr()
    owners = {}
    for k, p in enumerate(patches):
        for d in p.tolist():
            owners.setdefault(d, []).append(k)
    colour = {}
    for k in sorted(range(len(patches)), key=lambda k: (-len(patches[k]), k)):
        used = set()
        for d in np.unique(Kb[patches[k]].indices).tolist():
            for q in owners.get(d, ()):
                if q in colour:
                    used.add(colour[q])
        c = 0
        while c in used:
            c += 1
        colour[k] = c
    return [sorted(k for k in colour if colour[k] == c) for c in range(max(colour.values()) + 1)]


def patch_counts(n: int, patches) -> np.ndarray:
    """cnt(d): the number of patches that contain unknown d."""
    cnt = np.zeros(n, dtype=np.int64)
    for p in patches:
        cnt[p] += 1
    return cnt
