"""GPU parity of the symmetric panel layout of the patch inverses.

K_E is symmetric (Eq. intro_saddle with -D = G^T), so each patch inverse is
too; with CAV_LAYOUT_SYMMETRIC the library stores only its lower 16-column
panels (diagonal 16 x 16 blocks whole) and the additive smoother reads the
upper entries through their mirror images. The oracle still solves with LU
factors of the full patch matrices. The computed inverse is symmetric only up
to rounding (about kappa_1 2^-53 relative to its norm), so the smoother,
V-cycle and FGMRES keep the full layout's bounds against the oracle:
64 kappa_1 2^-53 for a sweep, four times that for a V-cycle, identical
FGMRES iteration counts, solution within 1e-8.
"""
import numpy as np
import pytest

import workloads
from oracle import krylov, multigrid

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ALPHA = 0.7
U = 2.0 ** -53
P = 16


def _solver():
    from paper_2608_14310_amd import Solver
    return Solver(0)


def _t(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def _np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _tol(fst):
    return max(1e-12, 64 * fst["max_cond"] * U)


def sym_size(n):
    """Stored entries of one n x n inverse in the panel layout: panel k holds
    rows 16k .. n-1 of columns 16k .. 16k + w - 1, w = min(16, n - 16k)."""
    return sum((n - k) * min(P, n - k) for k in range(0, n, P))


CASES = {
    "target32": lambda: workloads.small_target(0),
    "membrane32": lambda: workloads.membrane_ellipse(32, 3, 1e4, 1),
    "beam64": lambda: workloads.beam_fibres(64, 4, 1.0, 1e4, seed=0),
    "fibre64": lambda: workloads.flexible_fibre(64, 4, seed=0),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def spair(request):
    s = CASES[request.param]()
    print(f"[gpu symmetric] case {request.param} N={s.N} levels={s.n_levels}", flush=True)
    H = multigrid.Hierarchy(s, alpha=ALPHA)
    g = _solver()
    stats, fst = g.setup(s, alpha=ALPHA, layout="symmetric")
    yield request.param, s, H, g, stats, fst
    g.close()


def test_symmetric_sizes():
    # closed form of the panel arena against the count above
    for n in list(range(1, 70)) + [127, 128, 129, 178, 318]:
        t = -(-n // P)
        w = n - P * (t - 1)
        assert sym_size(n) == P * (t - 1) * n - 128 * (t - 1) * (t - 2) + w * w
        assert n * (n + 1) // 2 <= sym_size(n) <= n * (n + 1) // 2 + P * n // 2


def test_symmetric_factor_bytes(spair):
    """The stored bytes are those of the panel layout: per explicit patch
    sym_size(n) FP64 entries (explicit patches: the exported patches larger
    than the 5-unknown standard patch, plus any 5-unknown ones the level
    stats count)."""
    name, s, H, g, stats, fst = spair
    want = 0
    for l in range(1, s.n_levels):
        off, dofs = g.export_patches(l)
        ns = np.diff(off)
        big = ns[ns > 5]
        m5 = stats[l]["n_explicit"] - big.size
        assert int((big.astype(np.int64) ** 2).sum()) + 25 * m5 == stats[l]["sum_np2"], (name, l)
        want += 8 * (sum(sym_size(int(n)) for n in big) + m5 * sym_size(5))
    assert fst["factor_bytes"] == want, (fst["factor_bytes"], want)


def test_symmetric_sweep(spair):
    name, s, H, g, stats, fst = spair
    rng = np.random.default_rng(8)
    tol = _tol(fst)
    for l in range(1, len(H.levels)):
        b = rng.standard_normal(H.levels[l].K.shape[0])
        y = _np(g.level_apply(l, 3, _t(b)))
        ref = H.smooth(l, b, np.zeros_like(b))
        assert _rel(y, ref) < tol, (name, l, _rel(y, ref), tol)


def test_symmetric_vcycle(spair):
    name, s, H, g, stats, fst = spair
    z = _np(g.vcycle(_t(s.b)))
    assert _rel(z, H.vcycle(s.b)) < 4 * _tol(fst)


def test_symmetric_fgmres_matches_oracle(spair):
    name, s, H, g, stats, fst = spair
    K = H.levels[-1].K
    res = krylov.fgmres(lambda x: K @ x, H.vcycle, s.b, 1e-10, 150)
    x, info = g.fgmres_solve(_t(s.b), rtol=1e-10, max_it=150)
    xg = _np(x)
    print(f"[gpu symmetric] {name}: oracle its={res.iterations} gpu its={info['iterations']}", flush=True)
    assert info["converged"] == 1 and info["iterations"] == res.iterations
    assert np.linalg.norm(xg - res.x) / np.linalg.norm(res.x) < 1e-8
    np.testing.assert_allclose(info["history"], res.history, rtol=1e-5, atol=1e-13)


def test_symmetric_against_full_layout(spair):
    """Same system factored in both layouts: sweeps agree within the rounding
    bound of two explicit inverses."""
    name, s, H, g, stats, fst = spair
    f = _solver()
    try:
        _, ffst = f.setup(s, alpha=ALPHA)
        assert ffst["max_cond"] == fst["max_cond"]
        rng = np.random.default_rng(31)
        for l in range(1, s.n_levels):
            b = _t(rng.standard_normal(g.n(l)))
            a = _np(g.level_apply(l, 3, b))
            c = _np(f.level_apply(l, 3, b))
            assert _rel(a, c) < 2 * _tol(fst), (name, l, _rel(a, c))
            # colour phases, computed on demand under the symmetric layout
            pg, pf = g.export_phases(l), f.export_phases(l)
            assert pg == pf, (name, l)
    finally:
        f.close()


def test_multiplicative_needs_full_layout():
    """The multiplicative kernels read full inverses: over symmetric-layout
    factors they are refused (a clear error, nothing launched); after
    switching back to the full layout and factoring again they run and equal
    a context factored in the full layout from the start."""
    from paper_2608_14310_amd import CAVError
    s = CASES["beam64"]()
    g = _solver()
    ref = _solver()
    try:
        g.setup(s, alpha=1.0, layout="symmetric")
        g.set_smoother("multiplicative", 1.0)
        with pytest.raises(CAVError):
            g.vcycle(_t(s.b))
        with pytest.raises(CAVError):
            g.fgmres_solve(_t(s.b), rtol=1e-10, max_it=5)
        with pytest.raises(CAVError):
            g.autotune(reps=1)
        # a per-level override is refused the same way
        g.set_smoother("additive", 0.7)
        g.set_level_smoother(s.n_levels - 1, "multiplicative", 1.0)
        with pytest.raises(CAVError):
            g.vcycle(_t(s.b))
        g.set_level_smoother(s.n_levels - 1, None)
        z_add = _np(g.vcycle(_t(s.b)))
        assert np.isfinite(z_add).all()
        g.set_factor_layout("full")
        g.factor_patches("fp64", 1e6)
        g.set_smoother("multiplicative", 1.0)
        z = _np(g.vcycle(_t(s.b)))
        ref.setup(s, alpha=1.0, smoother="multiplicative")
        assert np.array_equal(z, _np(ref.vcycle(_t(s.b))))
    finally:
        g.close()
        ref.close()


def test_symmetric_mixed_precision():
    """FP32 panels for patches with kappa_1 <= 1e6: the V-cycle within the
    FP32 bound of the FP64 oracle's, FGMRES to 1e-10 with the solution within
    1e-8 of the oracle's."""
    s = CASES["beam64"]()
    H = multigrid.Hierarchy(s, alpha=ALPHA)
    g = _solver()
    try:
        stats, fst = g.setup(s, precision="mixed", cond_threshold=1e6, alpha=ALPHA, layout="symmetric")
        assert fst["n_fp32"] > 0
        z = _np(g.vcycle(_t(s.b)))
        tol = 64 * min(fst["max_cond"], 1e6) * 2.0 ** -24
        assert _rel(z, H.vcycle(s.b)) < tol
        K = H.levels[-1].K
        res = krylov.fgmres(lambda x: K @ x, H.vcycle, s.b, 1e-10, 150)
        x, info = g.fgmres_solve(_t(s.b), rtol=1e-10, max_it=150)
        xg = _np(x)
        print(f"[gpu symmetric] mixed beam64: its={info['iterations']} (fp64 oracle {res.iterations})", flush=True)
        assert info["converged"] == 1
        assert np.linalg.norm(s.b - K @ xg) / np.linalg.norm(s.b) < 2e-10
        assert np.linalg.norm(xg - res.x) / np.linalg.norm(res.x) < 1e-8
    finally:
        g.close()


def test_symmetric_box_family():
    """B(4,2) boxes (patches of up to 144 unknowns, restricted injection):
    the additive sweep over symmetric-layout factors against the oracle."""
    s = workloads.beam_fibres(64, 3, 1.0, 1e4, seed=0)
    H = multigrid.Hierarchy(s, alpha=ALPHA, family="box", box=(4, 2))
    g = _solver()
    try:
        stats, fst = g.setup(s, family="box", box=(4, 2), alpha=ALPHA, layout="symmetric")
        rng = np.random.default_rng(5)
        for l in range(1, s.n_levels):
            b = rng.standard_normal(H.levels[l].K.shape[0])
            y = _np(g.level_apply(l, 3, _t(b)))
            ref = H.smooth(l, b, np.zeros_like(b))
            assert _rel(y, ref) < _tol(fst), (l, _rel(y, ref))
    finally:
        g.close()
