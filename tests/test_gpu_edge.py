"""Edge cases, error paths and the full-size configuration on the GPU.

Degenerate systems (no markers, one marker, one level, the smallest grid),
zero and shifted right-hand sides against the oracle; invalid arguments and
out-of-order calls return the documented status codes; and the 512^2 beam
system that the benchmark times is checked by quantities the oracle computes
at that size: the finest-level E_E and patch sets exactly, K x, and the true
residual of the GPU solution evaluated with the oracle's own K_E.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads
from oracle import direct, ib, mac, multigrid, krylov
from oracle import patches as opatches

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cav():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    import paper_2608_14310_amd as cav
    cav.lib()
    return cav


def _t(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def _no_markers(N=16, levels=2):
    s = workloads.target_circle(N=N, n_levels=levels)
    return workloads.System("no_markers", N, levels, s.rho, s.mu, s.dt, "target", {"kappa_t": 1e4},
                            [workloads.Segment(np.zeros((0, 2)), True, 0.1)], s.b)


def _one_marker(N=16, levels=2):
    s = workloads.target_circle(N=N, n_levels=levels)
    seg = workloads.Segment(np.array([[0.37, 0.61]]), True, 0.5 / N)
    return workloads.System("one_marker", N, levels, s.rho, s.mu, s.dt, "target", {"kappa_t": 1e5}, [seg], s.b)


DEGENERATE = {
    "no_markers": lambda: _no_markers(),
    "one_marker": lambda: _one_marker(),
    "smallest_grid": lambda: workloads.target_circle(N=8, n_levels=2, kappa=1e4),
    "one_level": lambda: workloads.target_circle(N=8, n_levels=1, kappa=1e4),
}


@pytest.mark.parametrize("name", sorted(DEGENERATE))
@pytest.mark.parametrize("smoother,alpha,osm", [("additive", 0.7, "additive"), ("multiplicative", 1.0, "coloured")])
def test_degenerate_systems_match_oracle(cav, name, smoother, alpha, osm):
    s = DEGENERATE[name]()
    print(f"[edge] {name} {smoother}", flush=True)
    g = cav.Solver(0)
    g.setup(s, alpha=alpha, smoother=smoother)
    x, inf = g.fgmres_solve(_t(s.b), 1e-10, 60)
    g.close()
    H = multigrid.Hierarchy(s, alpha=alpha, smoother=osm)
    K = H.levels[-1].K
    ref = krylov.fgmres(lambda v: K @ v, H.vcycle, s.b, rtol=1e-10, max_it=60)
    assert inf["converged"] and ref.converged
    assert inf["iterations"] == ref.iterations, (inf["iterations"], ref.iterations)
    xs = direct.solve(K, s.N, s.b)
    xg = x.cpu().numpy()
    assert np.linalg.norm(xg - ref.x) <= 1e-8 * np.linalg.norm(ref.x)
    assert np.linalg.norm(K @ xg - s.b) <= 2e-10 * np.linalg.norm(s.b)
    if s.n_levels == 1:           # the coarse direct solve is the whole preconditioner
        assert inf["iterations"] == 1
        assert np.linalg.norm(xg - xs) <= 1e-9 * np.linalg.norm(xs)


def test_zero_and_shifted_rhs(cav):
    s = workloads.small_target()
    print("[edge] zero / shifted right-hand side", flush=True)
    g = cav.Solver(0)
    g.setup(s, alpha=0.7)
    x, inf = g.fgmres_solve(_t(np.zeros(s.n)), 1e-10, 50)
    assert inf["converged"] and inf["iterations"] == 0 and not x.abs().max().item()
    shift = 0.37
    b = s.b.copy()
    b[2 * s.N * s.N:] += shift                    # constant pressure: outside the range of K_E
    x1, i1 = g.fgmres_solve(_t(b), 1e-10, 50)
    x0, i0 = g.fgmres_solve(_t(s.b), 1e-10, 50)
    g.close()
    assert abs(i1["pressure_mean_removed"] - shift) < 1e-12
    assert i1["iterations"] == i0["iterations"]
    assert np.linalg.norm(x1.cpu().numpy() - x0.cpu().numpy()) <= 1e-12 * np.linalg.norm(x0.cpu().numpy())


def test_error_paths(cav):
    print("[edge] error paths", flush=True)
    from paper_2608_14310_amd import CAVError
    s = workloads.small_target()
    g = cav.Solver(0)
    r = torch.zeros(3 * 32 * 32, dtype=torch.float64, device="cuda")
    with pytest.raises(CAVError) as e:          # nothing built yet
        g.vcycle(r, out=torch.empty_like(r))
    assert e.value.status == 6
    bad = workloads.System("bad_N", 12, 2, s.rho, s.mu, s.dt, s.law, s.kappa, s.segments, np.zeros(3 * 144))
    with pytest.raises(CAVError) as e:
        g.build_operator(bad)
    assert e.value.status == 1
    deep = workloads.System("too_deep", 32, 5, s.rho, s.mu, s.dt, s.law, s.kappa, s.segments, s.b)
    with pytest.raises(CAVError) as e:
        g.build_operator(deep)
    assert e.value.status == 1
    nan_seg = workloads.Segment(np.array([[np.nan, 0.5]]), True, 0.01)
    nanx = workloads.System("nan_marker", 32, 3, s.rho, s.mu, s.dt, s.law, s.kappa, [nan_seg], s.b)
    with pytest.raises(CAVError) as e:
        g.build_operator(nanx)
    assert e.value.status == 1
    g.build_operator(s)
    with pytest.raises(CAVError) as e:          # patches not built / factored
        g.fgmres_solve(_t(s.b))
    assert e.value.status == 6
    g.build_cav_patches()
    g.factor_patches()
    with pytest.raises(CAVError) as e:
        g.fgmres_solve(_t(s.b), max_it=0)
    assert e.value.status == 1
    bnan = s.b.copy()
    bnan[5] = np.nan
    with pytest.raises(CAVError) as e:
        g.fgmres_solve(_t(bnan))
    assert e.value.status == 1
    with pytest.raises(CAVError) as e:          # learned stage requested without a net
        g.fgmres_solve(_t(s.b), learned=True)
    assert e.value.status == 6
    net = cav.Net(0)
    with pytest.raises(CAVError) as e:          # grid below the net's minimum
        net.forward(torch.zeros((1, 3, 4, 4), dtype=torch.float32, device="cuda"), 4)
    assert e.value.status == 1
    with pytest.raises(ValueError):
        net.set_weights(np.zeros(10, np.float32))
    net.close()
    x, inf = g.fgmres_solve(_t(s.b))           # the context still works after the errors
    assert inf["converged"]
    g.close()


def test_full_size_beam512(cav):
    """The benchmark's configuration, checked at full size: finest-level E_E
    and patch sets exactly, K x, the mixed-precision solution's true residual
    measured with the oracle's K_E, and bit-identical V-cycles and solves from
    every phase-kernel form. (The FP64 solve against the oracle's iteration
    count and solution is in test_gpu_golden.py.)"""
    s = workloads.beam_512(1e-2)
    print("[full size] beam512: oracle E_E and patches", flush=True)
    EE, pattern = ib.eulerian_elasticity(s)
    K = mac.reduced_operator(s.N, s.rho, s.mu, s.dt, EE)
    g = cav.Solver(0)
    stats, fst = g.setup(s, precision="mixed", alpha=1.0, smoother="multiplicative")
    top = s.n_levels - 1
    rp, col, val = g.export_ee(top)
    n = 2 * s.N * s.N
    G = sp.csr_matrix((val, col, rp), shape=(n, n))
    P = pattern.tocsr()
    assert np.array_equal(G.indptr, P.indptr) and np.array_equal(G.indices, P.indices)
    assert abs(G - EE).max() <= 1e-13 * abs(EE).max()
    ps, _ = opatches.cav_patches(s.N, pattern)
    off, dofs = g.export_patches(top)
    assert len(off) == len(ps) + 1
    for c, p in enumerate(ps):
        assert np.array_equal(dofs[off[c]:off[c + 1]], p), c
    print("[full size] beam512: K x and the solve", flush=True)
    xr = np.random.default_rng(3).standard_normal(K.shape[0])
    y = g.apply_operator(_t(xr)).cpu().numpy()
    assert np.abs(y - K @ xr).max() <= 1e-13 * np.abs(K @ xr).max()
    x, inf = g.fgmres_solve(_t(s.b), 1e-10, 150)
    print(f"[full size] beam512 mixed: {inf['iterations']} iterations", flush=True)
    assert inf["converged"]
    xg = x.cpu().numpy()
    assert np.linalg.norm(s.b - K @ xg) <= 2e-10 * np.linalg.norm(s.b)
    # the cooperative phase forms (large patches spread over several
    # workgroups) and the dataflow sweep give the same V-cycle bit for bit at
    # this size
    print("[full size] beam512: cooperative phase forms", flush=True)
    z0 = g.vcycle(_t(s.b)).cpu().numpy()
    for form, sweep in ((1, 0), (2, 0), (3, 0), (3, 2)):
        table = np.full((s.n_levels, 5), 1024, np.int32)
        table[:, 4] = sweep
        table[:, 2:4] = form
        g.set_tuning(table)
        np.testing.assert_array_equal(g.vcycle(_t(s.b)).cpu().numpy(), z0)
    x2, inf2 = g.fgmres_solve(_t(s.b), 1e-10, 150)
    g.close()
    assert inf2["iterations"] == inf["iterations"]
    np.testing.assert_array_equal(x2.cpu().numpy(), xg)


def test_barrier_wait_bound_reports_and_recovers(cav):
    """The cooperative phase kernels' barrier waits are bounded. A bound of
    zero polls forces the give-up path from the host: every kernel still
    finishes, the solve raises CAV_ERR_HIP, and with the bound restored the
    context solves again, bit for bit as before."""
    from paper_2608_14310_amd import CAVError
    s = workloads.beam_fibres(N=64, n_levels=4, kappa_b=1e-2)   # patches of up to 301 rows
    print("[edge] barrier wait bound", flush=True)
    g = cav.Solver(0)
    g.setup(s, precision="fp64", alpha=1.0, smoother="multiplicative")
    b = _t(s.b)
    x0, i0 = g.fgmres_solve(b, 1e-10, 150)
    g.set_wait_limit(0)
    with pytest.raises(CAVError) as e:
        g.fgmres_solve(b, 1e-10, 150)
    assert e.value.status == 3
    g.set_wait_limit()
    x1, i1 = g.fgmres_solve(b, 1e-10, 150)
    g.close()
    assert i1["converged"] and i1["iterations"] == i0["iterations"]
    np.testing.assert_array_equal(x1.cpu().numpy(), x0.cpu().numpy())


def test_setup_sequences_reproduce_a_fresh_context(cav):
    """The setup keeps work in flight between calls (coarsest factorisation
    started by build_operator, patch factorisations started by the patch
    build) and reuses released device memory. Every call sequence gives
    results bit-identical to a fresh context: patches rebuilt without a
    factorisation in between (pending work released), a second factorisation
    with another precision (coarsest inverse kept), a rebuilt operator of
    another system (everything restarted, memory reused), and back."""
    print("[edge] setup sequences", flush=True)
    sa = workloads.beam_fibres(64, 2, 1.0, 1e4, seed=0)
    sb = workloads.membrane_ellipse(32, 3, 1e4, 1)

    def fresh(s, precision):
        g = cav.Solver(0)
        g.setup(s, precision=precision, alpha=1.0, smoother="multiplicative")
        x, inf = g.fgmres_solve(_t(s.b), 1e-10, 150)
        z = g.vcycle(_t(s.b))
        torch.cuda.synchronize()
        out = (x.cpu().numpy(), z.cpu().numpy(), inf["iterations"])
        g.close()
        return out

    ref = {(s.name, p): fresh(s, p) for s in (sa, sb) for p in ("fp64", "mixed")}
    g = cav.Solver(0)

    def check(s, precision):
        x, inf = g.fgmres_solve(_t(s.b), 1e-10, 150)
        z = g.vcycle(_t(s.b))
        torch.cuda.synchronize()
        rx, rz, rits = ref[(s.name, precision)]
        assert inf["iterations"] == rits, (s.name, precision)
        assert np.array_equal(x.cpu().numpy(), rx), (s.name, precision)
        assert np.array_equal(z.cpu().numpy(), rz), (s.name, precision)

    g.build_operator(sa)
    g.build_cav_patches("cav")
    g.build_cav_patches("cav")                 # pending factorisations released, enqueued again
    g.factor_patches("fp64", 1e6)
    g.set_smoother("multiplicative", 1.0)
    check(sa, "fp64")
    g.factor_patches("mixed", 1e6)             # coarsest inverse kept, patches factored again
    g.set_smoother("multiplicative", 1.0)
    check(sa, "mixed")
    g.build_operator(sb)                       # another hierarchy: released memory reused
    g.build_cav_patches("cav")
    g.factor_patches("mixed", 1e6)
    g.set_smoother("multiplicative", 1.0)
    check(sb, "mixed")
    g.build_operator(sa)
    g.build_cav_patches("cav")
    g.factor_patches("fp64", 1e6)
    g.set_smoother("multiplicative", 1.0)
    check(sa, "fp64")
    g.close()


def test_kernel_timing_brackets(cav):
    """Live timing: brackets around runs of phase launches of one form; the
    shared-residual form is a part of the cooperative forms, which are a part
    of all phase launches; one top-level V-cycle is counted."""
    print("[edge] kernel timing", flush=True)
    s = workloads.beam_fibres(N=64, n_levels=4, kappa_b=1e-2)
    g = cav.Solver(0)
    g.setup(s, precision="fp64", alpha=1.0, smoother="multiplicative")
    # per-phase launches of the cooperative forms
    table = np.full((s.n_levels, 5), 3, np.int32)
    table[:, 4] = 0
    g.set_tuning(table)
    g.kernel_timing(True)
    g.vcycle(_t(s.b))
    kt = g.kernel_timing(False)
    assert kt["vcycles"] == 1 and kt["vcycle_ms"] > 0
    assert 0 < kt["shared_launches"] <= kt["coop_launches"] <= kt["launches"]
    assert 0 < kt["shared_ms"] <= kt["coop_ms"] <= kt["ms"]
    assert 0 < kt["shared_bytes"] <= kt["coop_bytes"] <= kt["bytes"]
    assert kt["flow_launches"] == 0
    phase_bytes = kt["bytes"]
    # the dataflow sweep: one launch per level sweep, the same algorithmic bytes
    table[:, 4] = 2
    g.set_tuning(table)
    g.kernel_timing(True)
    g.vcycle(_t(s.b))
    kt = g.kernel_timing(False)
    g.close()
    assert kt["coop_launches"] == 0 and 0 < kt["flow_launches"] == kt["launches"]
    assert 0 < kt["flow_ms"] <= kt["ms"]
    assert kt["flow_bytes"] == kt["bytes"] == phase_bytes


def test_kernel_timing_leaves_results_unchanged(cav):
    """Live timing brackets every weighted additive smoother launch with a pair
    of events and every top-level V-cycle with another; the solve with them is
    the solve without them, bit for bit, and every V-cycle counts one launch
    per smoothing step on each smoothed level."""
    print("[edge] kernel timing, additive V(3,3), symmetric layout", flush=True)
    s = workloads.beam_fibres(N=64, n_levels=4, kappa_b=1e-2)
    g = cav.Solver(0)
    g.setup(s, precision="fp64", alpha=0.9, layout="symmetric")
    g.set_smoother("additive", 0.9, 3, 3)
    b = _t(s.b)
    x0, i0 = g.fgmres_solve(b, rtol=1e-10, max_it=150)
    g.kernel_timing(True)
    x1, i1 = g.fgmres_solve(b, rtol=1e-10, max_it=150)
    kt = g.kernel_timing(False)
    g.close()
    assert i0["converged"] and i1["iterations"] == i0["iterations"]
    assert torch.equal(x0, x1)
    assert kt["vcycles"] > 0 and kt["vcycle_ms"] > 0 and kt["ms"] > 0 and kt["bytes"] > 0
    assert kt["launches"] == kt["vcycles"] * (s.n_levels - 1) * 6
