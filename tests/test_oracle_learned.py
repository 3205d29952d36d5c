"""Pins of the oracle's learned-correction stage (CPU only).

Each check ties the oracle to something other than itself: a library routine
for a special case (scipy's periodic correlation), exact algebraic properties
(translation equivariance, positive homogeneity, adjointness), central finite
differences for the gradient, closed forms of Adam's first steps, hand-derived
bfloat16 roundings, and the defining identities of the residual pairs and of
the stage's minimal-residual step.
"""
import numpy as np
import pytest
import scipy.ndimage as ndi

import workloads
from oracle import learned as L
from oracle import multigrid


def rand_weights(seed, scale=1.0):
    return np.random.default_rng(seed).uniform(-scale, scale, L.N_WEIGHTS)


def test_weight_count():
    assert L.N_WEIGHTS == 32 * 3 * 9 + 32 * 32 * 9 + 3 * 32 * 9 == 10944
    assert workloads.net_init(0).shape == (10944,)


def test_conv_matches_scipy_periodic_correlation():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3, 8, 8))
    W = rng.standard_normal((4, 3, 3, 3))
    y = L.conv(x, W)
    for b in range(2):
        for co in range(4):
            ref = sum(ndi.correlate(x[b, ci], W[co, ci], mode="wrap") for ci in range(3))
            np.testing.assert_allclose(y[b, co], ref, rtol=0, atol=1e-12)


def test_conv_single_tap_is_a_shift():
    # a weight with one tap at (a, c) reads x[i + a - 1, j + c - 1]
    x = np.arange(36.0).reshape(1, 1, 6, 6)
    for a in range(3):
        for c in range(3):
            W = np.zeros((1, 1, 3, 3))
            W[0, 0, a, c] = 1.0
            y = L.conv(x, W)[0, 0]
            for i in range(6):
                for j in range(6):
                    assert y[i, j] == x[0, 0, (i + a - 1) % 6, (j + c - 1) % 6]


def test_conv_transpose_is_adjoint():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 5, 7, 7))
    dy = rng.standard_normal((2, 4, 7, 7))
    W = rng.standard_normal((4, 5, 3, 3))
    lhs = np.sum(L.conv(x, W) * dy)
    rhs = np.sum(x * L.conv_transpose(dy, W))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))
    # the weight gradient is the derivative of <conv(x, W), dy> in W
    G = L.conv_weight_grad(dy, x)
    E = np.zeros_like(W)
    E[1, 2, 0, 2] = 1.0
    assert abs(np.sum(L.conv(x, E) * dy) - G[1, 2, 0, 2]) < 1e-12


def test_net_translation_equivariant_and_homogeneous():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((1, 3, 8, 8))
    w = rand_weights(4, 0.3)
    y, _ = L.forward(x, w)
    ys, _ = L.forward(np.roll(x, (2, -3), axis=(2, 3)), w)
    np.testing.assert_allclose(ys, np.roll(y, (2, -3), axis=(2, 3)), atol=1e-12)
    y2, _ = L.forward(4.0 * x, w)
    np.testing.assert_array_equal(y2, 4.0 * y)
    yb, _ = L.forward(-x, w)  # not odd: ReLU breaks the sign symmetry
    assert not np.allclose(yb, -y)


def test_bf16_rounding_hand_values():
    v = np.array([1.0 + 2 ** -8,            # tie -> even (1.0)
                  1.0 + 3 * 2 ** -8,        # tie -> even (1 + 2^-6)
                  -(1.0 + 2 ** -7 + 2 ** -9),  # below the midpoint -> 1 + 2^-7
                  1.0 + 2 ** -8 + 2 ** -20,   # above the midpoint -> 1 + 2^-7
                  2.0 ** -130, 0.0, 65504.0, 3.0])
    out = L.round_bf16(v)
    assert out[0] == 1.0
    assert out[1] == 1.0 + 2 ** -6
    assert out[2] == -(1.0 + 2 ** -7)
    assert out[3] == 1.0 + 2 ** -7
    assert out[5] == 0.0 and out[6] == 65536.0 and out[7] == 3.0
    # 8 significant bits: every result has at most 8 bits of mantissa
    m, _ = np.frexp(out[np.isfinite(out) & (out != 0)])
    assert np.all((m * 256) == np.round(m * 256))


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((2, 3, 6, 6))
    e = rng.standard_normal((2, 3, 6, 6))
    w = rand_weights(6, 0.4)
    _, g = L.loss_and_grad(x, e, w)
    picks = np.concatenate([rng.choice(864, 20, replace=False),
                            864 + rng.choice(9216, 30, replace=False),
                            864 + 9216 + rng.choice(864, 20, replace=False)])
    h = 1e-6
    for k in picks:
        wp, wm = w.copy(), w.copy()
        wp[k] += h
        wm[k] -= h
        fd = (L.loss_and_grad(x, e, wp)[0] - L.loss_and_grad(x, e, wm)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_residual_loss_gradient_matches_central_differences():
    s = workloads.target_circle(N=8, n_levels=1)
    from oracle import ib, mac
    EE, _ = ib.eulerian_elasticity(s)
    K = mac.reduced_operator(s.N, s.rho, s.mu, s.dt, EE)
    assert abs(K - K.T).max() < 1e-9 * abs(K).max()      # K_E is symmetric (G = -D^T, E_E symmetric)
    rng = np.random.default_rng(9)
    x = rng.standard_normal((2, 3, 8, 8))
    w = rand_weights(10, 0.4)
    loss, g = L.residual_loss_and_grad(x, K, w)
    # direct evaluation of the definition
    y, _ = L.forward(x, w)
    direct = np.mean([np.sum((K @ y[b].ravel() - x[b].ravel()) ** 2) / np.sum(x[b] ** 2) for b in range(2)])
    assert abs(loss - direct) <= 1e-12 * direct
    picks = np.concatenate([rng.choice(864, 12, replace=False), 864 + rng.choice(9216, 20, replace=False),
                            864 + 9216 + rng.choice(864, 12, replace=False)])
    h = 1e-6
    for k in picks:
        wp, wm = w.copy(), w.copy()
        wp[k] += h
        wm[k] -= h
        fd = (L.residual_loss_and_grad(x, K, wp)[0] - L.residual_loss_and_grad(x, K, wm)[0]) / (2 * h)
        # the loss is large (K carries rho/dt = 1e3), so the difference quotient's
        # rounding error is eps * loss / h, about 1e-5 of the derivative here
        assert abs(fd - g[k]) <= 1e-4 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_minres_loss_definition_and_gradient():
    s = workloads.target_circle(N=8, n_levels=1)
    from oracle import ib, mac
    EE, _ = ib.eulerian_elasticity(s)
    K = mac.reduced_operator(s.N, s.rho, s.mu, s.dt, EE)
    rng = np.random.default_rng(12)
    x = rng.standard_normal((2, 3, 8, 8))
    w = rand_weights(13, 0.4)
    loss, g = L.minres_loss_and_grad(x, K, w)
    # definition: the residual left by the best multiple, found by a scalar least-squares fit
    y, _ = L.forward(x, w)
    direct = []
    for b in range(2):
        kc, r = K @ y[b].ravel(), x[b].ravel()
        gam = np.linalg.lstsq(kc[:, None], r, rcond=None)[0][0]
        direct.append(np.sum((r - gam * kc) ** 2) / np.sum(r ** 2))
    assert abs(loss - np.mean(direct)) <= 1e-10
    assert 0.0 <= loss <= 1.0
    # scale invariance: scaling the output layer leaves the loss unchanged
    w2 = w.copy()
    w2[864 + 9216:] *= 8.0
    assert abs(L.minres_loss_and_grad(x, K, w2)[0] - loss) <= 1e-12
    picks = np.concatenate([rng.choice(864, 12, replace=False), 864 + rng.choice(9216, 20, replace=False),
                            864 + 9216 + rng.choice(864, 12, replace=False)])
    h = 1e-6
    for k in picks:
        wp, wm = w.copy(), w.copy()
        wp[k] += h
        wm[k] -= h
        fd = (L.minres_loss_and_grad(x, K, wp)[0] - L.minres_loss_and_grad(x, K, wm)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1e-3, abs(g[k])), (k, fd, g[k])


def test_loss_normalisation():
    rng = np.random.default_rng(7)
    x = rng.standard_normal((3, 3, 4, 4))
    e = rng.standard_normal((3, 3, 4, 4))
    loss, g = L.loss_and_grad(x, e, np.zeros(L.N_WEIGHTS))
    assert abs(loss - 1.0) < 1e-15          # zero network: every sample scores 1
    assert np.all(g == 0.0)                  # and ReLU(0) passes no gradient


def test_adam_first_steps_closed_form():
    opt = L.Adam(lr=1e-3)
    w0 = np.array([0.5, -0.25, 1.0, 0.0])
    g1 = np.array([2.0, -1e-3, 0.0, 5.0])
    w1, st = opt.step(w0, g1, opt.init(4))
    # step 1: m_hat = g, v_hat = g^2 -> update lr g / (|g| + eps)
    np.testing.assert_allclose(w1, w0 - 1e-3 * g1 / (np.abs(g1) + 1e-8), rtol=0, atol=1e-18)
    g2 = np.array([-2.0, 3e-3, 1.0, 5.0])
    w2, _ = opt.step(w1, g2, st)
    m = 0.9 * 0.1 * g1 + 0.1 * g2
    v = 0.999 * 0.001 * g1 ** 2 + 0.001 * g2 ** 2
    ref = w1 - 1e-3 * (m / (1 - 0.81)) / (np.sqrt(v / (1 - 0.999 ** 2)) + 1e-8)
    np.testing.assert_allclose(w2, ref, rtol=1e-14, atol=1e-18)


@pytest.fixture(scope="module")
def small_target_setup():
    s = workloads.target_circle(N=16, n_levels=2)
    h = multigrid.Hierarchy(s, family="cav", alpha=1.0, smoother="multiplicative")
    K = h.levels[-1].K
    return s, h, K


def test_residual_pairs_identity(small_target_setup):
    s, h, K = small_target_setup
    xs = workloads.random_solutions(s.N, 1, 0)[0]
    pairs = L.residual_pairs(K, h.vcycle, xs, 3)
    prev = None
    for r, e in pairs:
        assert abs(np.linalg.norm(r) - 1.0) < 1e-14
        np.testing.assert_allclose(K @ e, r, atol=1e-9)      # K e_k = r_k
        n = np.linalg.norm(e)
        assert prev is None or n > 0
        prev = n


def test_stage_gamma_is_the_minimiser(small_target_setup):
    s, h, K = small_target_setup
    rng = np.random.default_rng(8)
    direction = rng.standard_normal(K.shape[0])
    stage = L.LearnedStage(K, h.vcycle, lambda rh: direction, s.N, margin=0.0)
    v = rng.standard_normal(K.shape[0])
    z = stage(v)
    z0 = h.vcycle(v)
    c = L.remove_pressure_mean(np.linalg.norm(v - K @ z0) * direction, s.N)
    # z - z0 is gamma c; gamma must beat every other multiple of c
    gamma = float((z - z0) @ c / (c @ c))
    res = lambda t: np.linalg.norm(v - K @ (z0 + t * c))
    for t in np.linspace(gamma - 1, gamma + 1, 41):
        assert res(gamma) <= res(t) + 1e-12


def test_stage_exact_corrector_one_iteration(small_target_setup):
    s, h, K = small_target_setup
    from oracle import direct, krylov
    exact = lambda rh: direct.solve(K, s.N, rh)
    stage = L.LearnedStage(K, h.vcycle, exact, s.N)
    res = krylov.fgmres(lambda x: K @ x, stage, s.b, rtol=1e-10, max_it=20)
    assert res.converged and res.iterations <= 2 and stage.accepted >= 1


def test_stage_zero_weights_rejected(small_target_setup):
    s, h, K = small_target_setup
    from oracle import krylov
    stage = L.LearnedStage(K, h.vcycle, L.net_corrector(np.zeros(L.N_WEIGHTS), s.N), s.N)
    res = krylov.fgmres(lambda x: K @ x, stage, s.b, rtol=1e-10, max_it=60)
    plain = krylov.fgmres(lambda x: K @ x, h.vcycle, s.b, rtol=1e-10, max_it=60)
    assert stage.accepted == 0 and stage.rejected == res.iterations
    assert res.iterations == plain.iterations
