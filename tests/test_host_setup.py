"""Host logic of the HIP library against the oracle, on the CPU.

cav_analyze runs the host part of the setup (force law, E_E = S E J,
Galerkin coarsening, CAV patches, multiplicative colour phases, 1/cnt
weights) with no device; every result must equal the oracle's: patch sets
and phases exactly, E_E to rounding.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads
from oracle import ib, hierarchy, mac, multigrid, patches as pmod


def _analysis(s, family="cav"):
    from paper_2608_14310_amd._binding import Analysis
    return Analysis(s, family)


CASES = {
    "target32": lambda: workloads.small_target(0),
    "membrane32": lambda: workloads.membrane_ellipse(32, 3, 1e4, 1),
    "beam64": lambda: workloads.beam_fibres(64, 4, 1.0, 1e4, seed=0),
    "closedbeam32": lambda: workloads.paper_beam(32),
    "fibre64": lambda: workloads.flexible_fibre(64, 4, seed=0),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def pair(request):
    s = CASES[request.param]()
    a = _analysis(s)
    EE, pat = ib.eulerian_elasticity(s)
    ee = [None] * s.n_levels
    ee[-1] = (EE, pat)
    for l in range(s.n_levels - 1, 0, -1):
        ee[l - 1] = hierarchy.galerkin(ee[l][0], ee[l][1], s.N >> (s.n_levels - l))
    yield request.param, s, a, ee
    a.close()


def test_library_exports_every_declared_symbol():
    """Every function include/cavmg.h declares is exported by libcavmg.so."""
    import os
    import re
    import ctypes
    from paper_2608_14310_amd import library_path
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "cavmg.h")).read()
    names = set(re.findall(r"\b(cav_[a-z_0-9]+)\s*\(", hdr))
    L = ctypes.CDLL(library_path())
    missing = [n for n in sorted(names) if not hasattr(L, n)]
    assert names and not missing, missing


def test_ee_matches_oracle(pair):
    name, s, a, ee = pair
    for l in range(s.n_levels):
        rp, col, val = a.ee(l)
        N = s.N >> (s.n_levels - 1 - l)
        G = sp.csr_matrix((val, col, rp), shape=(2 * N * N, 2 * N * N))
        EE, pat = ee[l]
        P = pat.tocsr()
        assert np.array_equal(np.diff(G.indptr), np.diff(P.indptr)), (name, l)
        assert np.array_equal(G.indices, P.indices), (name, l)
        d = (G - EE).tocsr()
        assert (abs(d).max() if d.nnz else 0.0) <= 1e-13 * max(abs(EE).max(), 1e-300), (name, l)


def test_patches_phases_and_weights_match_oracle(pair):
    name, s, a, ee = pair
    for l in range(1, s.n_levels):
        N = s.N >> (s.n_levels - 1 - l)
        ps, std = pmod.cav_patches(N, ee[l][1])
        got = a.patches(l)
        assert len(got) == len(ps)
        assert all(np.array_equal(g, p) for g, p in zip(got, ps)), (name, l)
        stencil = mac.reduced_operator(N, 1.0, 1.0, 1.0, sp.csr_matrix((2 * N * N, 2 * N * N)))
        want = pmod.coloured_order(N, ps, ee[l][1], stencil)
        ph = a.phases(l)
        assert ph == want[:len(ph)], (name, l)
        cnt = pmod.patch_counts(3 * N * N, ps)
        dofs, inv = a.weights(l)
        assert np.array_equal(inv, 1.0 / cnt[dofs]), (name, l)
        # every unknown outside the touched list sits in exactly the standard count of patches
        rest = np.setdiff1d(np.arange(3 * N * N), dofs)
        assert np.all(cnt[rest[rest < 2 * N * N]] == 2) and np.all(cnt[rest[rest >= 2 * N * N]] == 1)


def test_vanka_family_is_standard():
    s = workloads.small_target(0)
    a = _analysis(s, "vanka")
    for l in range(1, s.n_levels):
        N = s.N >> (s.n_levels - 1 - l)
        got = a.patches(l)
        assert all(len(p) == 5 for p in got)
        assert all(np.array_equal(g, pmod.vanka_patch(N, c // N, c % N)) for c, g in enumerate(got))


@pytest.mark.parametrize("name", ["membrane32", "beam64"])
def test_box_family_matches_oracle(name):
    """B(4,2) boxes (Section 3.1): dof sets exactly, colour phases equal to the
    oracle's coloured box order (seed cells = block lower-left cells), and the
    injected-slot lists: each unknown receives exactly the boxes whose
    unexpanded block holds it, with weight 1."""
    from paper_2608_14310_amd._binding import Analysis
    s = CASES[name]()
    a = Analysis(s, "box", (4, 2))
    EE, pat = ib.eulerian_elasticity(s)
    ee = [None] * s.n_levels
    ee[-1] = (EE, pat)
    for l in range(s.n_levels - 1, 0, -1):
        ee[l - 1] = hierarchy.galerkin(ee[l][0], ee[l][1], s.N >> (s.n_levels - l))
    for l in range(1, s.n_levels):
        N = s.N >> (s.n_levels - 1 - l)
        ps, inj = pmod.box_patches(N, 4, 2)
        seeds = [I * N + J for I in range(0, N, 4) for J in range(0, N, 4)]
        got = a.patches(l)
        for c in range(N * N):
            if c in seeds:
                assert np.array_equal(got[c], ps[seeds.index(c)]), (name, l, c)
            else:
                assert len(got[c]) == 0
        stencil = mac.reduced_operator(N, 1.0, 1.0, 1.0, sp.csr_matrix((2 * N * N, 2 * N * N)))
        want = [[seeds[k] for k in ph] for ph in pmod.coloured_box_order(N, ps, ee[l][1], stencil)]
        assert a.phases(l) == want, (name, l)
        dofs, inv = a.weights(l)
        cnt = np.zeros(3 * N * N, dtype=int)
        for p, m in zip(ps, inj):
            cnt[p[m]] += 1
        assert np.array_equal(dofs, np.nonzero(cnt)[0]) and np.all(inv == 1.0)
        assert np.all(cnt > 0)                      # the blocks cover every unknown
    a.close()


def test_box_oracle_sweeps_are_consistent():
    """The oracle's coloured box sweep equals its lexicographic box sweep in the
    coloured order (same patches, same injection), and phases are independent:
    applying a phase's boxes in reverse order gives the same result."""
    from oracle import smoothers
    s = CASES["membrane32"]()
    H = multigrid.Hierarchy(s, family="box", alpha=1.0, smoother="coloured")
    l = s.n_levels - 1
    lev = H.levels[l]
    b = np.random.default_rng(4).standard_normal(lev.K.shape[0])
    x = H.smooth(l, b, np.zeros_like(b))
    rev = [k for ph in lev.phases for k in reversed(ph)]
    sol = smoothers.PatchSolvers(lev.K, [lev.patches[k] for k in rev], lev.standard[rev], [lev.inject[k] for k in rev])
    x2 = smoothers.multiplicative_sweep(lev.K, sol, b, np.zeros_like(b), lev.N, [lev.inject[k] for k in rev])
    assert np.abs(x - x2).max() <= 1e-12 * np.abs(x).max()


@pytest.mark.parametrize("bad", ["clamp_low", "clamp_high", "closed", "two_segments"])
def test_fibre_law_rejects_invalid_structures(bad):
    """The fibre law (Section 5.3) needs one open segment with the clamp marker
    strictly inside it; anything else is an argument error, not a crash."""
    import dataclasses
    from paper_2608_14310_amd import CAVError
    s = workloads.flexible_fibre(32, 2, seed=0)
    M = len(s.segments[0].X)
    if bad == "clamp_low":
        s.kappa = dict(s.kappa, m=0)
    elif bad == "clamp_high":
        s.kappa = dict(s.kappa, m=M - 1)
    elif bad == "closed":
        s.segments = [dataclasses.replace(s.segments[0], closed=True)]
    else:
        seg = s.segments[0]
        s.segments = [dataclasses.replace(seg, X=seg.X[:M // 2]), dataclasses.replace(seg, X=seg.X[M // 2:])]
    with pytest.raises(CAVError):
        _analysis(s)


def test_fibre_force_matches_oracle():
    """The library's host force of the fibre law (Section 5.3) against the
    oracle's, at the markers and at a displaced configuration (X_force)."""
    from oracle import fibre, newton
    from paper_2608_14310_amd import structure_force
    s = workloads.flexible_fibre(64, 4, amp=0.3, seed=2)
    p = newton.fibre_params(s)
    X = s.markers().ravel()
    for Xf in (None, X + np.random.default_rng(9).uniform(-0.3, 0.3, X.shape) * p["ds"]):
        F = structure_force(s, Xf)
        ref = fibre.force(X if Xf is None else Xf, p)
        assert np.abs(F - ref).max() <= 1e-12 * np.abs(ref).max()
    with pytest.raises(Exception):
        structure_force(workloads.small_target(0))


def test_fibre_tangent_at_x_force_matches_oracle():
    """With X_force the fibre's tangent is taken there while J and S stay at
    the markers (Section 2: S and J at the start of the step, the force at the
    new configuration): finest E_E = S E(X_force) J against the oracle."""
    from oracle import fibre, newton
    from paper_2608_14310_amd._binding import Analysis
    s = workloads.flexible_fibre(64, 3, amp=0.2, seed=3)
    p = newton.fibre_params(s)
    X = s.markers().ravel()
    Xf = X + np.random.default_rng(4).uniform(-0.4, 0.4, X.shape) * p["ds"]
    a = Analysis(s, X_force=Xf)
    try:
        rp, col, val = a.ee(s.n_levels - 1)
    finally:
        a.close()
    n = 2 * s.N * s.N
    G = sp.csr_matrix((val, col, rp), shape=(n, n))
    J = ib.interpolation(s.N, s.markers())
    S = ib.spreading(s.N, J, s.weights())
    ref = (S @ fibre.tangent(Xf, p) @ J).tocsr()
    d = (G - ref).tocsr()
    assert abs(d).max() <= 1e-13 * abs(ref).max()
    # and it differs from the tangent at the markers
    a0 = Analysis(s)
    try:
        rp0, col0, val0 = a0.ee(s.n_levels - 1)
    finally:
        a0.close()
    G0 = sp.csr_matrix((val0, col0, rp0), shape=(n, n))
    assert abs(G0 - G).max() > 1e-6 * abs(ref).max()


def test_fibre_force_with_incremental_links():
    """The library's force at X + X_disp forms the links incrementally
    (Section 5.3): on a nearly straight fibre at 256^2 it agrees with an
    extended-precision evaluation to about 1e-12 of its size, where the
    absolute-position form (X_force = X + X_disp) loses two more digits; carried
    links equal to the markers' differences give the same force, and the
    oracle's incremental force agrees."""
    import dataclasses
    import fibre_extended
    from oracle import fibre, newton
    from paper_2608_14310_amd import structure_force
    s0 = workloads.flexible_fibre(256, 2)
    p = newton.fibre_params(s0)
    Xn, disp = fibre_extended.straight_fibre_step(s0)
    seg = dataclasses.replace(s0.segments[0], X=Xn.reshape(-1, 2))
    s = dataclasses.replace(s0, segments=[seg])
    ref = fibre_extended.force(Xn, disp, p)
    scale = np.abs(ref).max()
    F = structure_force(s, X_disp=disp)
    assert np.abs(F - ref).max() <= 5e-12 * scale
    Fa = structure_force(s, X_force=Xn + disp)
    assert np.abs(Fa - ref).max() >= 20 * np.abs(F - ref).max()
    X2 = Xn.reshape(-1, 2)
    Fl = structure_force(s, X_disp=disp, links=(X2[1:] - X2[:-1]).ravel())
    assert np.array_equal(Fl, F)
    d2 = disp.reshape(-1, 2)
    Fo = fibre.force(Xn + disp, p, D=(X2[1:] - X2[:-1]) + (d2[1:] - d2[:-1]))
    assert np.abs(F - Fo).max() <= 1e-12 * scale
    with pytest.raises(Exception):
        structure_force(s, X_disp=np.full_like(disp, np.nan))
