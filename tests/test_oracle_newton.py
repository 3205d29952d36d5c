"""Pins of the oracle's Newton step for the fibre (Section 2 scheme, Section 5.3).

* The Newton matrix K_E (E = tangent at the current configuration, S and J at
  X^n) is the derivative of the residual R: central differences of R along
  random directions.
* A straight fibre exactly at its clamp, at rest, with no load is an
  equilibrium: R(0) = 0 and no correction is taken.
* With every stiffness zero the force vanishes and one correction is the
  Stokes solve (a library LU of K_0), after which the residual is at rounding.
* Exact Newton converges quadratically: r_{k+1} / r_k^2 stays bounded over the
  last corrections of a strongly nonlinear step.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads
from oracle import direct, newton


def _step(N=32, amp=0.3, seed=1, dt_factor=1.0):
    s = workloads.flexible_fibre(N, 3, amp=amp, seed=seed)
    s.dt = s.dt * dt_factor
    un = workloads.fibre_inflow_velocity(N, seed=seed)
    rhs = np.concatenate([s.rho / s.dt * un, np.zeros(N * N)])
    return s, rhs


def test_jacobian_is_the_derivative_of_the_residual():
    s, rhs = _step(16, dt_factor=20.0)
    st = newton.Step(s)
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, 3 * s.N * s.N)
    K = st.jacobian(x)
    for _ in range(3):
        v = rng.uniform(-1, 1, x.size)
        eps = 1e-5
        fd = (st.residual(x + eps * v, rhs) - st.residual(x - eps * v, rhs)) / (2 * eps)
        Kv = K @ v
        assert np.linalg.norm(fd - Kv) <= 1e-7 * np.linalg.norm(Kv)
    # the elastic part alone (without K_0) also matches, so the tangent is not hidden by the fluid terms
    v = rng.uniform(-1, 1, x.size)
    eps = 1e-5
    fd = (st.residual(x + eps * v, rhs) - st.residual(x - eps * v, rhs)) / (2 * eps) - st.K0 @ v
    el = (K - st.K0) @ v
    assert np.linalg.norm(el) > 0
    assert np.linalg.norm(fd - el) <= 1e-5 * np.linalg.norm(el)


def test_straight_clamped_fibre_at_rest_is_an_equilibrium():
    s, _ = _step(32)
    seg = s.segments[0]
    M = len(seg.X)
    m = s.kappa["m"]
    X = np.stack([0.5 + (np.arange(M) - m) * seg.ds, np.full(M, 0.75)], axis=1)
    s.segments = [type(seg)(X, False, seg.ds)]
    rhs = np.zeros(3 * s.N * s.N)
    r = newton.solve(s, rhs)
    assert r.residuals[0] == 0.0 and r.corrections == 0 and r.converged
    np.testing.assert_array_equal(r.X, X.ravel())


def test_zero_stiffness_is_one_stokes_solve():
    s, rhs = _step(32)
    s.kappa = dict(s.kappa, EI=0.0, K_s=0.0, K_p=0.0, K_t=0.0)
    r = newton.solve(s, rhs)
    assert r.corrections == 1 and r.converged
    st = newton.Step(s)
    B = direct.bordered(st.K0, s.N)
    ref = spla.splu(B).solve(np.concatenate([rhs, [0.0]]))[:-1]
    assert np.linalg.norm(r.x - ref) <= 1e-12 * np.linalg.norm(ref)
    assert r.residuals[1] <= 1e-12 * r.residuals[0]


def test_exact_newton_converges_quadratically():
    s, rhs = _step(32, dt_factor=20.0)
    r = newton.solve(s, rhs, rtol=1e-14, atol=0.0, max_newton=6)
    res = r.residuals
    assert r.corrections >= 4
    q = [res[k + 1] / res[k] ** 2 for k in range(len(res) - 1) if res[k + 1] > 1e-11 * res[0]]
    tail = q[-2:]
    assert len(tail) == 2 and max(tail) / min(tail) < 10.0, res
