"""Pins of the flexible-fibre energies, force and tangent (Section 5.3).

The oracle's gradient and Hessian are checked against central differences of
the energy and of the gradient, against the invariances of the bending and
stretching energies (rigid translations and rotations change neither), and
against closed forms at the straight reference configuration."""
import numpy as np
import pytest

import workloads
from oracle import fibre



def _params(M, ds):
    return dict(ds=ds, EI=2.63672e-2, K_s=375.0, K_p=1200.0, K_t=7.03125, m=M // 2, Xc=np.array([0.5, 0.75]))


def _bent(M=13, ds=1.0 / 128, amp=0.3, seed=0):
    rng = np.random.default_rng(seed)
    s = (np.arange(M) - M // 2) * ds
    X = np.stack([0.5 + s, 0.75 - amp * s ** 2 / (M * ds)], axis=1)
    X += rng.uniform(-0.05, 0.05, X.shape) * ds
    return X.ravel(), _params(M, ds)


def test_gradient_matches_central_differences():
    x, p = _bent()
    g = fibre.gradient(x, p)
    eps = 1e-7 * p["ds"]
    fd = np.array([(fibre.energy(x + eps * e, p) - fibre.energy(x - eps * e, p)) / (2 * eps)
                   for e in np.eye(x.size)])
    assert np.abs(g - fd).max() <= 1e-5 * np.abs(g).max()


def test_hessian_matches_central_differences_of_the_gradient():
    x, p = _bent()
    H = fibre.hessian(x, p).toarray()
    eps = 1e-7 * p["ds"]
    fd = np.stack([(fibre.gradient(x + eps * e, p) - fibre.gradient(x - eps * e, p)) / (2 * eps)
                   for e in np.eye(x.size)], axis=1)
    assert np.abs(H - fd).max() <= 1e-5 * np.abs(H).max()
    assert np.array_equal(H, H.T)


def test_tangent_is_minus_hessian_over_ds_and_couples_components():
    x, p = _bent()
    E = fibre.tangent(x, p)
    assert np.allclose(E.toarray(), -fibre.hessian(x, p).toarray() / p["ds"], rtol=0, atol=0)
    assert np.abs(E.toarray()[0::2, 1::2]).max() > 0          # x-y coupling
    M = x.size // 2
    assert E.nnz == 4 * sum(min(M, i + 3) - max(0, i - 2) for i in range(M))   # fixed banded-block pattern
    # force = -(1/ds) grad energy, and its derivative is the tangent
    eps = 1e-7 * p["ds"]
    e = np.random.default_rng(1).standard_normal(x.size)
    dF = (fibre.force(x + eps * e, p) - fibre.force(x - eps * e, p)) / (2 * eps)
    assert np.abs(dF - E @ e).max() <= 1e-5 * np.abs(E @ e).max()


def test_bending_and_stretching_are_rigid_motion_invariant():
    x, p = _bent()
    G = fibre.gradient(x, p, parts=("b", "s")).reshape(-1, 2)
    X = x.reshape(-1, 2)
    scale = np.abs(G).max()
    assert np.abs(G.sum(axis=0)).max() <= 1e-10 * scale * len(X)            # translations
    assert abs(np.sum(X[:, 0] * G[:, 1] - X[:, 1] * G[:, 0])) <= 1e-10 * scale * len(X)   # rotations
    H = fibre.hessian(x, p, parts=("b", "s")).toarray()
    tx = np.tile([1.0, 0.0], len(X))
    assert np.abs(H @ tx).max() <= 1e-9 * np.abs(H).max()


def test_straight_reference_configuration_closed_forms():
    """Straight fibre along x at rest length: no bending or stretching force;
    the stretching Hessian is K_s/ds D1^T D1 on the x components and zero on
    y; the bending Hessian is EI/ds^5 grad(c) grad(c)^T (c = 0), whose y-y
    block is EI/ds^3 D2^T D2; the tangent is negative semidefinite."""
    M, ds = 11, 1.0 / 64
    p = _params(M, ds)
    s = (np.arange(M) - M // 2) * ds
    X = np.stack([0.5 + s, np.full(M, 0.75)], axis=1)
    x = X.ravel()
    assert np.abs(fibre.gradient(x, p, parts=("b", "s"))).max() <= 1e-12
    D1 = np.diff(np.eye(M), axis=0)
    D2 = np.diff(np.eye(M), n=2, axis=0)
    Hs = fibre.hessian(x, p, parts=("s",)).toarray()
    assert np.allclose(Hs[0::2, 0::2], p["K_s"] / ds * D1.T @ D1, rtol=1e-12, atol=1e-9)
    assert np.abs(Hs[1::2, 1::2]).max() <= 1e-9 and np.abs(Hs[0::2, 1::2]).max() <= 1e-9
    Hb = fibre.hessian(x, p, parts=("b",)).toarray()
    assert np.allclose(Hb[1::2, 1::2], p["EI"] / ds ** 3 * D2.T @ D2, rtol=1e-12, atol=1e-6)
    assert np.abs(Hb[0::2, 0::2]).max() <= 1e-9
    ev = np.linalg.eigvalsh(fibre.tangent(x, p).toarray())
    assert ev.max() <= 1e-9 * np.abs(ev).max()


def test_penalties_closed_forms():
    x, p = _bent()
    m = p["m"]
    Hp = fibre.hessian(x, p, parts=("p",)).toarray()
    assert np.allclose(Hp[2 * m:2 * m + 2, 2 * m:2 * m + 2], p["K_p"] * np.eye(2)) and np.count_nonzero(Hp) == 2
    Ht = fibre.hessian(x, p, parts=("t",)).toarray()
    k = p["K_t"] / (4 * p["ds"] ** 2)
    assert np.allclose(Ht[2 * (m + 1), 2 * (m - 1)], -k) and np.allclose(Ht[2 * (m - 1), 2 * (m - 1)], k)


def test_workload_has_the_papers_marker_counts():
    """The fibre workload puts the paper's number of markers on each grid of
    Section 5.3, Table 3 (length 0.375 at ds = h/2 in the paper's cell)."""
    import os
    import workloads
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_table3.txt")
    rows = [line.split() for line in open(path) if line.strip() and not line.startswith("#")]
    assert len(rows) == 4
    for r in rows:
        s = workloads.flexible_fibre(int(r[0]), 3)
        assert len(s.markers()) == int(r[1])
        assert s.kappa["m"] == int(r[1]) // 2


def test_workload_parameters_map_the_papers_values():
    """On the 128² grid (the paper's 128 x 128 grid, h = 1/64 in its cell) the
    fibre's parameters are the paper's (Section 5.3) mapped by the length
    scale 1/2: EI s^3, K_s s, K_p, K_t s^2, mu s; they double per halving of
    h, and Table 4's factors multiply them."""
    import workloads
    s = workloads.flexible_fibre(128, 5)
    k = s.kappa
    assert np.isclose(k["EI"] * 8, 2.63672e-2) and np.isclose(k["K_s"] * 2, 375.0)
    assert np.isclose(k["K_p"], 1200.0) and np.isclose(k["K_t"] * 4, 7.03125)
    assert np.isclose(s.mu * 2, 1.875e-3) and np.isclose(s.dt, 0.05 / 128)
    s2 = workloads.flexible_fibre(256, 6)
    assert np.isclose(s2.kappa["K_s"], 2 * k["K_s"]) and np.isclose(s2.kappa["EI"], k["EI"])
    s3 = workloads.flexible_fibre(128, 5, Re=2000.0, gamma=(10.0, 0.1, 10.0))
    assert np.isclose(s3.mu, s.mu / 10) and np.isclose(s3.kappa["EI"], 10 * k["EI"])
    assert np.isclose(s3.kappa["K_s"], 0.1 * k["K_s"]) and np.isclose(s3.kappa["K_t"], 10 * k["K_t"])
    # Reynolds number rho U L / mu with U = 1 and the scaled length 0.1875
    assert np.isclose(1.0 * 1.0 * 0.1875 / s.mu, 200.0)


def test_incremental_links_keep_the_bending_force_of_a_straight_fibre():
    """Section 5.3 updates the links incrementally. On a nearly straight fibre
    at 256^2 (ds = h/2) after one step's displacement, the force with links
    D^n + (disp_{k+1} - disp_k) agrees with an extended-precision evaluation
    to about 1e-12 of its size, while differences of the rounded absolute
    positions lose two more digits (their error grows like ds^-4)."""
    import fibre_extended
    s = workloads.flexible_fibre(256, 2)
    from oracle import newton
    p = newton.fibre_params(s)
    Xn, disp = fibre_extended.straight_fibre_step(s)
    ref = fibre_extended.force(Xn, disp, p)
    X2, d2 = Xn.reshape(-1, 2), disp.reshape(-1, 2)
    D = (X2[1:] - X2[:-1]) + (d2[1:] - d2[:-1])
    scale = np.abs(ref).max()
    err_incr = np.abs(fibre.force(Xn + disp, p, D=D) - ref).max() / scale
    err_abs = np.abs(fibre.force(Xn + disp, p) - ref).max() / scale
    assert err_incr <= 5e-12, err_incr
    assert err_abs >= 20 * err_incr, (err_abs, err_incr)      # the fixture does exercise the cancellation
