"""cav_fgmres_solve_noalloc (the FGMRES entry point for callers that cannot
allocate) against cav_fgmres_solve, through the C ABI.

Both entry points run the same kernels in the same order on the same inputs,
so the iteration counts and residual histories must be identical and the
solutions equal within the FP64 parity bar (1e-12 relative; in practice bit
for bit). Two calls in a row share the device's fixed scratch: the second
solves a smaller system, so it runs over what the first left behind.
"""
import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

INVALID_ARG = 1


def _t(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def _compare(g, b, smoother, alpha, label):
    g.set_smoother(smoother, alpha)
    x_ref = g.empty()
    x_na = g.empty()
    x_na.fill_(np.nan)
    _, ref = g.fgmres_solve(b, rtol=1e-10, max_it=150, out=x_ref)
    _, na = g.fgmres_solve(b, rtol=1e-10, max_it=150, out=x_na, noalloc=True)
    torch.cuda.synchronize()
    a, r = x_na.cpu().numpy(), x_ref.cpu().numpy()
    rel = np.abs(a - r).max() / np.abs(r).max()
    print(f"[noalloc] {label} {smoother}: its {na['iterations']} / {ref['iterations']}, "
          f"max rel diff {rel:.2e}, bitwise {np.array_equal(a, r)}", flush=True)
    assert na["status"] == ref["status"] == 0, (na["status"], ref["status"])
    assert na["iterations"] == ref["iterations"]
    assert np.array_equal(na["history"], ref["history"])
    assert na["true_rel_residual"] <= 2e-10
    assert rel <= 1e-12, rel


def test_noalloc_matches_allocating_solve_twice_smaller_second():
    from paper_2608_14310_amd import Solver
    g = Solver(0)
    try:
        big = workloads.membrane_ellipse(64, 4, 1e4, 1)
        print(f"[noalloc] case membrane64 N={big.N}", flush=True)
        g.setup(big, alpha=0.7)
        b = _t(big.b)
        _compare(g, b, "multiplicative", 1.0, "membrane64")
        small = workloads.small_target(0)
        print(f"[noalloc] case target32 N={small.N}", flush=True)
        g.setup(small, alpha=0.7)
        # noalloc first this time, over the scratch the 64^2 solves left behind
        g.set_smoother("additive", 0.7)
        bs = _t(small.b)
        x_na = g.empty()
        _, na = g.fgmres_solve(bs, rtol=1e-10, max_it=150, out=x_na, noalloc=True)
        x_ref = g.empty()
        _, ref = g.fgmres_solve(bs, rtol=1e-10, max_it=150, out=x_ref)
        torch.cuda.synchronize()
        a, r = x_na.cpu().numpy(), x_ref.cpu().numpy()
        rel = np.abs(a - r).max() / np.abs(r).max()
        print(f"[noalloc] target32 additive: its {na['iterations']} / {ref['iterations']}, max rel diff {rel:.2e}",
              flush=True)
        assert na["iterations"] == ref["iterations"] and na["status"] == ref["status"] == 0
        assert np.array_equal(na["history"], ref["history"])
        assert rel <= 1e-12, rel
    finally:
        g.close()


def test_noalloc_rejects_oversized_and_learned_requests():
    from paper_2608_14310_amd import Solver
    from paper_2608_14310_amd._binding import CAVError
    g = Solver(0)
    try:
        s = workloads.membrane_ellipse(64, 4, 1e4, 1)
        g.setup(s, alpha=0.7)
        b = _t(s.b)
        x = g.empty()
        # (2 * 10000 + 3) vectors of 3 * 64^2 doubles exceed the 512 MiB scratch
        with pytest.raises(CAVError) as e:
            g.fgmres_solve(b, rtol=1e-10, max_it=10000, out=x, noalloc=True)
        assert e.value.status == INVALID_ARG and "bytes" in str(e.value)
        with pytest.raises(CAVError) as e:
            g.fgmres_solve(b, rtol=1e-10, max_it=20, out=x, noalloc=True, learned=True)
        assert e.value.status == INVALID_ARG
        # the context still solves afterwards
        _, info = g.fgmres_solve(b, rtol=1e-10, max_it=150, out=x, noalloc=True)
        assert info["status"] == 0
    finally:
        g.close()
