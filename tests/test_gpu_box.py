"""B(b,o) box family with restricted injection on the GPU (Section 3.1, 3.3).

Against the oracle's box family: one smoother sweep and the V-cycle to the
V-cycle parity bound (explicit inverses against LU solves: 64 kappa_1 u per
sweep, floor 1e-12), and FGMRES with the same iteration count and solution
(1e-8), for the additive sweep (sum of injected corrections) and the coloured
multiplicative sweep (boxes in colour phases, injection on update).
"""
import numpy as np
import pytest

import workloads
from oracle import krylov, multigrid

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U = 2.0 ** -53


def _t(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


CASES = {"membrane32": lambda: workloads.membrane_ellipse(32, 3, 1e4, 1),
         "beam64": lambda: workloads.beam_fibres(64, 4, 1e-2, 1e4, seed=0)}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("smoother,osm,alpha", [("additive", "additive", 1.0), ("multiplicative", "coloured", 1.0)])
def test_box_family_matches_oracle(name, smoother, osm, alpha):
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    from paper_2608_14310_amd import Solver
    s = CASES[name]()
    print(f"[box family] {name} {smoother}", flush=True)
    H = multigrid.Hierarchy(s, family="box", alpha=alpha, smoother=osm, box=(4, 2))
    g = Solver(0)
    stats, fst = g.setup(s, family="box", alpha=alpha, smoother=smoother, box=(4, 2))
    assert stats[-1]["n_patches"] == (s.N // 4) ** 2
    tol = max(1e-12, 64 * fst["max_cond"] * U)
    rng = np.random.default_rng(5)
    for l in range(1, s.n_levels):
        b = rng.standard_normal(H.levels[l].K.shape[0])
        y = g.level_apply(l, 3, _t(b)).cpu().numpy()
        ref = H.smooth(l, b, np.zeros_like(b))
        assert _rel(y, ref) < tol, (l, _rel(y, ref), tol)
    z = g.vcycle(_t(s.b)).cpu().numpy()
    assert _rel(z, H.vcycle(s.b)) < 4 * tol
    K = H.levels[-1].K
    res = krylov.fgmres(lambda v: K @ v, H.vcycle, s.b, 1e-10, 150)
    x, inf = g.fgmres_solve(_t(s.b), 1e-10, 150)
    g.close()
    print(f"[box family] {name} {smoother}: oracle its={res.iterations} gpu its={inf['iterations']}", flush=True)
    assert inf["converged"] == res.converged and inf["iterations"] == res.iterations
    if res.converged:
        assert np.linalg.norm(x.cpu().numpy() - res.x) <= 1e-8 * np.linalg.norm(res.x)
    else:   # both stall (additive box smoothing on the beam): the same residual history
        np.testing.assert_allclose(inf["history"][:30], np.asarray(res.history)[:30], rtol=1e-6)
