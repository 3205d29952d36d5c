"""GPU parity of the learned correction stage against the float64 oracle.

Tolerances. The kernels round weights, inputs and hidden activations to
bfloat16 exactly where the oracle does; they differ only in summing in FP32
(order and precision) instead of float64, plus the rare activation whose FP32
and float64 sums straddle a bfloat16 rounding boundary (one bf16 ulp, 2^-8
relative, on that activation). Per output element the error is therefore
bounded by a small multiple of 2^-8 times the sum of the absolute values of the
terms that make it (the "abs bound", computed by the oracle on |W| and |a|);
norm-wise it stays near the FP32 level. The thresholds below (2^-8 x abs bound
per element, 2^-10 norm-wise) keep a factor of 30 or more over what an FP32
emulation of the same arithmetic shows, while any indexing mistake gives
errors of order one.
"""
import numpy as np
import pytest

import workloads
from oracle import krylov, learned as L, multigrid

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    return torch.device("cuda", 0)


@pytest.fixture(scope="module")
def cav():
    import paper_2608_14310_amd as cav
    cav.lib()
    return cav


def check_field(gpu, orc, bound, what):
    d = np.abs(gpu - orc)
    rel = np.linalg.norm(gpu - orc) / max(np.linalg.norm(orc), 1e-300)
    assert rel <= 2.0 ** -10, f"{what}: norm-wise relative error {rel:.3e}"
    worst = np.max(d - 2.0 ** -8 * bound)
    assert worst <= 1e-30, f"{what}: element beyond 2^-8 x abs bound by {worst:.3e}"


@pytest.mark.parametrize("N,B", [(8, 1), (16, 3), (32, 2), (64, 1)])
def test_forward_parity(dev, cav, N, B):
    print(f"[net forward] N={N} B={B}", flush=True)
    w = workloads.net_init(N)
    rng = np.random.default_rng(N)
    x = rng.standard_normal((B, 3, N, N)).astype(np.float32)
    net = cav.Net(0, w)
    y = net.forward(torch.from_numpy(x).to(dev), N).cpu().numpy().astype(np.float64)
    net.close()
    yo, c = L.forward(x.astype(np.float64), w.astype(np.float64), bf16=True)
    bound = L.conv(np.abs(c.a2), np.abs(c.Ws[2]))
    check_field(y, yo, bound, "y3")


def test_correct_parity(dev, cav):
    N = 32
    print(f"[net correct] N={N}", flush=True)
    w = workloads.net_init(7)
    r = np.random.default_rng(3).uniform(-1e-3, 1e-3, 3 * N * N)
    net = cav.Net(0, w)
    c = net.correct(torch.from_numpy(r).to(dev), N).cpu().numpy()
    zero = net.correct(torch.zeros(3 * N * N, dtype=torch.float64, device=dev), N).cpu().numpy()
    net.close()
    nr = np.linalg.norm(r)
    yo, cc = L.forward(L.to_image(r / nr, N)[None], w.astype(np.float64), bf16=True)
    co = L.remove_pressure_mean(nr * yo[0].ravel(), N)
    bound = nr * L.conv(np.abs(cc.a2), np.abs(cc.Ws[2]))[0].ravel()
    # the pressure-mean removal adds at most the mean of the element errors
    check_field(c, co, bound + 2.0 ** -8 * np.mean(bound[2 * N * N:]), "c")
    assert np.abs(c[2 * N * N:].mean()) < 1e-15 * nr * 3 * N * N
    assert np.all(zero == 0.0)


def test_train_step_parity(dev, cav):
    N, B = 16, 4
    print(f"[net train step] N={N} B={B}", flush=True)
    rng = np.random.default_rng(11)
    ns = 6
    rh = rng.standard_normal((ns, 3, N, N)).astype(np.float32)
    eh = rng.standard_normal((ns, 3, N, N)).astype(np.float32)
    idx = np.array([5, 0, 3, 2], dtype=np.int32)
    w0 = workloads.net_init(2)
    net = cav.Net(0, w0)
    lr = 1e-3
    loss = net.train_step(torch.from_numpy(rh.reshape(ns, -1)).to(dev), torch.from_numpy(eh.reshape(ns, -1)).to(dev),
                          N, idx, lr)
    w1, g = net.weights()
    net.close()
    lo, go = L.loss_and_grad(rh[idx].astype(np.float64), eh[idx].astype(np.float64), w0.astype(np.float64), bf16=True)
    assert abs(loss - lo) <= 2.0 ** -10 * lo
    for name, sl in (("dW1", slice(0, 864)), ("dW2", slice(864, 864 + 9216)), ("dW3", slice(864 + 9216, None))):
        gg, oo = g[sl].astype(np.float64), go[sl]
        rel = np.linalg.norm(gg - oo) / np.linalg.norm(oo)
        assert rel <= 2.0 ** -9, f"{name}: norm-wise relative error {rel:.3e}"
        assert np.max(np.abs(gg - oo)) <= 2.0 ** -7 * np.max(np.abs(oo)), name
    # first Adam step: the update is -lr g/(|g| + eps), i.e. -lr sign(g) where |g| >> eps;
    # the FP32 master weight rounds the result to half an ulp of w
    dw = w1.astype(np.float64) - w0.astype(np.float64)
    slack = lr * 1e-6 + 2.0 ** -24 * np.abs(w0.astype(np.float64)) * 2
    assert np.all(np.abs(dw) <= lr + slack)
    sure = np.abs(go) >= 2.0 ** -6 * np.max(np.abs(go))
    assert np.all(np.abs(dw[sure] + lr * np.sign(go[sure])) <= slack[sure])


@pytest.fixture(scope="module")
def target16():
    s = workloads.target_circle(N=32, n_levels=3)
    h = multigrid.Hierarchy(s, family="cav", alpha=1.0, smoother="coloured")
    return s, h, h.levels[-1].K


def _solver(cav, s):
    g = cav.Solver(0)
    g.setup(s, precision="fp64", alpha=1.0, smoother="multiplicative")
    return g


def test_learned_pairs_parity(dev, cav, target16):
    s, h, K = target16
    print(f"[learned pairs] N={s.N}", flush=True)
    xs = workloads.random_solutions(s.N, 2, 0)
    g = _solver(cav, s)
    rh, eh = g.learned_pairs(torch.from_numpy(xs).to(dev), iters=3)
    g.close()
    rh, eh = rh.cpu().numpy().astype(np.float64), eh.cpu().numpy().astype(np.float64)
    q = 0
    for x in xs:
        for r, e in L.residual_pairs(K, h.vcycle, x, 3):
            # FP32 storage of the pair; the V-cycle parity error is far smaller
            np.testing.assert_allclose(rh[q], r, rtol=0, atol=2.0 ** -22 * np.max(np.abs(r)))
            np.testing.assert_allclose(eh[q], e, rtol=0, atol=2.0 ** -22 * np.max(np.abs(e)))
            q += 1


def test_fgmres_stage_zero_net_rejects_everything(dev, cav, target16):
    s, h, K = target16
    print(f"[learned stage, zero net] N={s.N}", flush=True)
    g = _solver(cav, s)
    net = cav.Net(0, np.zeros(10944, dtype=np.float32))
    g.attach_net(net, margin=1e-3)
    b = torch.from_numpy(s.b).to(dev)
    _, plain = g.fgmres_solve(b, rtol=1e-10, max_it=60)
    _, inf = g.fgmres_solve(b, rtol=1e-10, max_it=60, learned=True)
    g.close()
    net.close()
    assert inf["learned_accepted"] == 0 and inf["learned_rejected"] == inf["iterations"]
    assert inf["iterations"] == plain["iterations"] and inf["converged"]
    np.testing.assert_array_equal(inf["history"], plain["history"])


def test_fgmres_stage_matches_oracle(dev, cav, target16):
    """margin 0: every correction is taken; iteration counts match the oracle's
    stage to within one (the corrections differ at the bf16 level) and both reach
    1e-10 with the same solution."""
    s, h, K = target16
    print(f"[learned stage vs oracle] N={s.N}", flush=True)
    w = workloads.net_init(5)
    g = _solver(cav, s)
    net = cav.Net(0, w)
    g.attach_net(net, margin=0.0)
    x, inf = g.fgmres_solve(torch.from_numpy(s.b).to(dev), rtol=1e-10, max_it=60, learned=True)
    x = x.cpu().numpy()
    g.close()
    net.close()
    stage = L.LearnedStage(K, h.vcycle, L.net_corrector(w.astype(np.float64), s.N), s.N, margin=0.0)
    res = krylov.fgmres(lambda v: K @ v, stage, s.b, rtol=1e-10, max_it=60)
    assert inf["converged"] and res.converged
    assert abs(inf["iterations"] - res.iterations) <= 1
    assert inf["learned_accepted"] == inf["iterations"] and stage.accepted == res.iterations
    err = np.linalg.norm(x - res.x) / np.linalg.norm(res.x)
    assert err < 1e-8, err


@pytest.mark.parametrize("kind", ["residual", "minres"])
def test_train_step_through_operator_parity(dev, cav, kind):
    s = workloads.target_circle(N=16, n_levels=2)
    print(f"[net train step through K] kind={kind} N={s.N}", flush=True)
    from oracle import ib, mac
    EE, _ = ib.eulerian_elasticity(s)
    K = mac.reduced_operator(s.N, s.rho, s.mu, s.dt, EE)
    rng = np.random.default_rng(21)
    ns, N = 5, s.N
    rh = rng.standard_normal((ns, 3 * N * N)).astype(np.float32)
    idx = np.array([4, 1, 2], dtype=np.int32)
    w0 = workloads.net_init(3, out_scale=1e-2)
    g = cav.Solver(0)
    g.build_operator(s)
    net = cav.Net(0, w0)
    loss = g.train_net_residual(net, torch.from_numpy(rh).to(dev), idx, 1e-3, kind)
    _, grad = net.weights()
    g.close()
    net.close()
    f = L.residual_loss_and_grad if kind == "residual" else L.minres_loss_and_grad
    lo, go = f(rh[idx].reshape(3, 3, N, N).astype(np.float64), K, w0.astype(np.float64), bf16=True)
    assert abs(loss - lo) <= 2.0 ** -10 * abs(lo), (loss, lo)
    for name, sl in (("dW1", slice(0, 864)), ("dW2", slice(864, 864 + 9216)), ("dW3", slice(864 + 9216, None))):
        gg, oo = grad[sl].astype(np.float64), go[sl]
        rel = np.linalg.norm(gg - oo) / np.linalg.norm(oo)
        assert rel <= 2.0 ** -9, f"{name}: norm-wise relative error {rel:.3e}"


def test_learned_gain_and_enable_rule(dev, cav):
    """Trains the net on V-cycle pairs of a 64^2 membrane system (minimal-residual
    loss) and measures what the stage gains inside FGMRES on held-out
    right-hand sides; the stage is enabled only where it cuts iterations."""
    from paper_2608_14310_amd import learned as LN
    s = workloads.membrane_ellipse(N=64, kappa=1e4)
    print(f"[learned gain] {s.name}", flush=True)
    g = _solver(cav, s)
    xs = torch.from_numpy(workloads.random_solutions(s.N, 100, 1)).to(dev)
    rh, eh = LN.generate_pairs(g, xs, 3)
    net = cav.Net(0, workloads.net_init(0, out_scale=1e-2))
    losses = LN.train(net, rh, eh, s.N, workloads.batch_order(rh.shape[0], 8, 600, 0), 1e-3, solver=g, kind="minres")
    rhs = [torch.from_numpy(workloads.random_rhs(s.N, 100 + k)).to(dev) for k in range(2)]
    enabled, rows = LN.validate(g, net, rhs)
    print(f"[learned gain] loss {np.mean(losses[:20]):.3f} -> {np.mean(losses[-50:]):.3f}; "
          f"iterations plain/learned {[(r['plain'], r['learned']) for r in rows]}; enabled={enabled}", flush=True)
    assert np.mean(losses[-50:]) < np.mean(losses[:20])       # training reduces the loss
    assert all(r["plain_converged"] and r["learned_converged"] for r in rows)
    assert enabled == all(r["learned"] < r["plain"] for r in rows)
    # a disabled stage leaves the solver on the plain V-cycle
    _, inf = g.fgmres_solve(rhs[0], 1e-10, 150, learned=enabled)
    assert inf["iterations"] == (rows[0]["learned"] if enabled else rows[0]["plain"])
    g.close()
    net.close()
