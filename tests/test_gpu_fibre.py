"""The flexible-fibre law (Section 5.3) through the whole device path.

A Newton solve of the clamped fibre rebuilds the hierarchy for every linear
system, each at a new fibre configuration. One context is set up for a
sequence of such iterates (straight to strongly bent), and every solve is
checked against the oracle: FGMRES iteration counts equal to the oracle's
(additive smoother, same cycle), solutions against the oracle's direct
solve. At 256² the multiplicative cycle's solution is checked by its true
residual under the oracle's operator.
"""
import numpy as np
import pytest

import workloads
from oracle import direct, ib, krylov, mac, multigrid

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _t(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def _oracle_K(s):
    EE, _ = ib.eulerian_elasticity(s)
    return mac.reduced_operator(s.N, s.rho, s.mu, s.dt, EE)


def test_newton_iterates_rebuild_in_one_context():
    from paper_2608_14310_amd import Solver
    g = Solver(0)
    try:
        for amp, seed in [(0.0, 1), (0.15, 2), (0.3, 3)]:
            s = workloads.flexible_fibre(64, 4, amp=amp, seed=seed)
            print(f"[fibre] iterate amp={amp} seed={seed} N=64", flush=True)
            K = _oracle_K(s)
            xd = direct.solve(K, s.N, s.b)
            H = multigrid.Hierarchy(s, alpha=0.7)
            res = krylov.fgmres(lambda v: K @ v, H.vcycle, s.b, 1e-10, 150)
            g.setup(s, alpha=0.7)
            x, info = g.fgmres_solve(_t(s.b), rtol=1e-10, max_it=150)
            torch.cuda.synchronize()
            xg = x.cpu().numpy()
            assert info["converged"] == 1 and info["iterations"] == res.iterations, (amp, info["iterations"],
                                                                                   res.iterations)
            assert np.linalg.norm(xg - xd) / np.linalg.norm(xd) < 1e-8
            g.setup(s, alpha=1.0, smoother="multiplicative")
            x, info = g.fgmres_solve(_t(s.b), rtol=1e-10, max_it=150)
            torch.cuda.synchronize()
            xg = x.cpu().numpy()
            print(f"[fibre] additive its={res.iterations} multiplicative its={info['iterations']}", flush=True)
            assert info["converged"] == 1
            assert np.linalg.norm(xg - xd) / np.linalg.norm(xd) < 1e-8
    finally:
        g.close()


def test_fibre_256_multiplicative_true_residual():
    from paper_2608_14310_amd import Solver
    s = workloads.flexible_fibre(256, 6, amp=0.3, seed=4)
    print("[fibre] N=256 levels=6 multiplicative", flush=True)
    g = Solver(0)
    try:
        g.setup(s, alpha=1.0, smoother="multiplicative")
        x, info = g.fgmres_solve(_t(s.b), rtol=1e-10, max_it=150)
        torch.cuda.synchronize()
        xg = x.cpu().numpy()
    finally:
        g.close()
    K = _oracle_K(s)
    true = np.linalg.norm(s.b - K @ xg) / np.linalg.norm(s.b)
    floor = direct.rounding_floor(K, xg, s.b)
    print(f"[fibre] its={info['iterations']} est={info['est_rel_residual']:.3e} true={true:.3e}", flush=True)
    assert info["converged"] == 1
    assert true <= 2 * max(1e-10, 10 * floor)
    assert abs(true - info["true_rel_residual"]) <= 1e-2 * true + 10 * floor
    assert abs(xg[2 * s.N * s.N:].mean()) < 1e-9 * np.abs(xg).max()


def test_interpolation_and_spreading_match_oracle():
    from paper_2608_14310_amd import Solver
    s = workloads.flexible_fibre(64, 4, amp=0.3, seed=5)
    print("[fibre] interpolation / spreading N=64", flush=True)
    J = ib.interpolation(s.N, s.markers())
    S = ib.spreading(s.N, J, s.weights())
    rng = np.random.default_rng(6)
    n2 = s.N * s.N
    x = rng.uniform(-1, 1, 3 * n2)
    F = rng.uniform(-1, 1, J.shape[0])
    y0 = rng.uniform(-1, 1, 3 * n2)
    g = Solver(0)
    try:
        g.build_operator(s)
        U = g.ib_interpolate(_t(x)).cpu().numpy()
        y = g.ib_spread_add(_t(F), _t(y0)).cpu().numpy()
    finally:
        g.close()
    Uo = J @ x[:2 * n2]
    assert np.abs(U - Uo).max() <= 1e-13 * np.abs(Uo).max()
    yo = y0.copy()
    yo[:2 * n2] += S @ F
    assert np.abs(y - yo).max() <= 1e-13 * np.abs(yo).max()
    assert np.array_equal(y[2 * n2:], y0[2 * n2:])


@pytest.mark.parametrize("N,levels,Re,gamma", [(64, 4, 200.0, (1.0, 1.0, 1.0)), (128, 5, 200.0, (1.0, 1.0, 1.0)),
                                               (64, 4, 2000.0, (10.0, 10.0, 10.0)),
                                               (64, 4, 200.0, (0.1, 1.0, 1.0))])
def test_newton_step_matches_oracle(N, levels, Re, gamma):
    """One backward-Euler step of the fibre in the downward stream by Newton's
    method: every correction rebuilds the hierarchy on the GPU and solves with
    multiplicative-CAV FGMRES to 1e-9; the oracle solves every Newton system
    directly. Same number of corrections, same solution; baseline parameters
    and two of Table 4's extreme rows."""
    from oracle import newton
    from paper_2608_14310_amd import Solver
    s = workloads.flexible_fibre(N, levels, amp=0.3, seed=1, Re=Re, gamma=gamma)
    un = workloads.fibre_inflow_velocity(N, seed=1)
    rhs = np.concatenate([s.rho / s.dt * un, np.zeros(N * N)])
    print(f"[fibre] Newton step N={N} levels={levels} Re={Re} gamma={gamma}", flush=True)
    ref = newton.solve(s, rhs, rtol=1e-8, atol=1e-8, max_newton=10)
    g = Solver(0)
    try:
        x, Xn, info = g.newton_solve(s, _t(rhs), rtol=1e-8, atol=1e-8, max_newton=10, lin_rtol=1e-9)
        torch.cuda.synchronize()
        xg = x.cpu().numpy()
    finally:
        g.close()
    print(f"[fibre] oracle corrections={ref.corrections} residuals={['%.3e' % r for r in ref.residuals]}; "
          f"gpu corrections={info['newton_its']} res0={info['res0']:.3e} res={info['res']:.3e} "
          f"fgmres total={info['fgmres_its_total']} max={info['fgmres_its_max']}", flush=True)
    assert ref.converged and info["converged"] == 1
    assert info["newton_its"] == ref.corrections
    assert abs(info["res0"] - ref.residuals[0]) <= 1e-12 * ref.residuals[0]
    assert info["res"] <= 1e-8 * info["res0"]
    assert np.linalg.norm(xg - ref.x) <= 1e-7 * np.linalg.norm(ref.x)
    assert np.abs(Xn - ref.X).max() <= 1e-12


def test_newton_edge_cases():
    """No correction allowed: the initial residual is reported and the step is
    flagged unconverged; a law other than the fibre is an argument error; two
    identical steps in one context give bit-identical results."""
    from paper_2608_14310_amd import CAVError, Solver
    s = workloads.flexible_fibre(32, 3, amp=0.3, seed=2)
    un = workloads.fibre_inflow_velocity(32, seed=2)
    rhs = _t(np.concatenate([s.rho / s.dt * un, np.zeros(32 * 32)]))
    print("[fibre] Newton edge cases N=32", flush=True)
    g = Solver(0)
    try:
        x, Xn, info = g.newton_solve(s, rhs, max_newton=0)
        assert info["newton_its"] == 0 and info["converged"] == 0 and info["res"] == info["res0"] > 0
        assert info["status"] != 0
        with pytest.raises(CAVError):
            g.newton_solve(workloads.small_target(0), rhs)
        x1, X1, i1 = g.newton_solve(s, rhs)
        x2, X2, i2 = g.newton_solve(s, rhs)
        torch.cuda.synchronize()
        assert i1["converged"] == 1 and i1 == i2
        assert torch.equal(x1, x2) and np.array_equal(X1, X2)
    finally:
        g.close()


def test_newton_with_capped_linear_solves_reports_every_field():
    """lin_max_it = 1: no Newton system's FGMRES meets lin_rtol, yet each
    correction is applied (inexact Newton) and counted as unconverged; the
    info fields and X_new are filled whatever the final status."""
    from paper_2608_14310_amd import Solver
    s = workloads.flexible_fibre(32, 3, amp=0.3, seed=2)
    un = workloads.fibre_inflow_velocity(32, seed=2)
    rhs = _t(np.concatenate([s.rho / s.dt * un, np.zeros(32 * 32)]))
    print("[fibre] Newton with lin_max_it=1 N=32", flush=True)
    g = Solver(0)
    try:
        x, Xn, info = g.newton_solve(s, rhs, max_newton=4, lin_max_it=1)
        torch.cuda.synchronize()
        print(f"[fibre] capped Newton info {info}", flush=True)
        assert info["status"] in (0, 100)
        assert info["newton_its"] >= 1 and info["failed_stage"] == 0
        assert info["lin_unconverged"] == info["newton_its"]
        assert info["fgmres_its_max"] == 1 and info["fgmres_its_total"] == info["newton_its"]
        assert np.isfinite(info["res"]) and info["res0"] > 0 and info["res"] < info["res0"]
        assert info["converged"] == (1 if info["status"] == 0 else 0)
        # X_new is the configuration of the last iterate: X^n + dt J^n u
        U = g.ib_interpolate(x).cpu().numpy()
        X0 = s.markers().ravel()
        assert np.abs(Xn - (X0 + s.dt * U)).max() <= 1e-14 * max(1.0, np.abs(X0).max())
    finally:
        g.close()
