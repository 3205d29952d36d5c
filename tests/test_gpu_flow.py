"""The dataflow form of the multiplicative sweep against the per-phase launches.

The dataflow launch runs a level's explicit phases in one kernel, each patch
starting once its conflicting predecessors of earlier colours are done. Patches
that do not conflict commute, so every V-cycle and every FGMRES solve must
equal the per-phase form bit for bit, over many consecutive sweeps (the
counters are monotonic across launches), in both phase orders, with FP32
factors, and with the box family's restricted injection.
"""
import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _t(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


CASES = {
    "beam64": (lambda: workloads.beam_fibres(64, 4, 1e-2, 1e4, seed=0), "cav", "fp64", "explicit_first"),
    "beam64_mixed_stdfirst": (lambda: workloads.beam_fibres(64, 4, 1.0, 1e4, seed=2), "cav", "mixed",
                              "standard_first"),
    "membrane64_box": (lambda: workloads.membrane_ellipse(64, 4, 1e4, 1), "box", "fp64", "explicit_first"),
    "fibre64": (lambda: workloads.flexible_fibre(64, 4, seed=0), "cav", "fp64", "explicit_first"),
}


def _table(n_levels, mode):
    t = np.full((n_levels, 5), 3, np.int32)
    t[:, 4] = mode
    return t


@pytest.mark.parametrize("name", sorted(CASES))
def test_flow_sweep_equals_phase_launches(name):
    from paper_2608_14310_amd import Solver
    make, family, precision, order = CASES[name]
    s = make()
    print(f"[flow] {name} N={s.N}", flush=True)
    g = Solver(0)
    try:
        g.setup(s, family=family, precision=precision, alpha=1.0, smoother="multiplicative")
        g.set_phase_order(order)
        b = _t(s.b)
        rng = np.random.default_rng(7)
        rs = [_t(rng.standard_normal(s.n)) for _ in range(4)]
        out = {}
        for mode in (2, 0, 2):
            g.set_tuning(_table(s.n_levels, mode))
            g.kernel_timing(True)
            zs = [g.vcycle(r).cpu().numpy() for r in rs for _ in range(3)]
            kt = g.kernel_timing(False)
            x, inf = g.fgmres_solve(b, rtol=1e-10, max_it=150)
            torch.cuda.synchronize()
            if mode == 2:
                assert kt["flow_launches"] > 0 and kt["shared_launches"] == 0, kt
            else:
                assert kt["flow_launches"] == 0 and kt["shared_launches"] > 0, kt
            cur = (zs, x.cpu().numpy(), inf["iterations"])
            if mode in out:
                ref = out[mode]
            else:
                ref = out.get(2)
                out[mode] = cur
            if ref is not None:
                for za, zb in zip(cur[0], ref[0]):
                    np.testing.assert_array_equal(za, zb)
                np.testing.assert_array_equal(cur[1], ref[1])
                assert cur[2] == ref[2]
        assert inf["converged"] == 1
    finally:
        g.close()


def test_flow_sweep_timing_and_grid():
    """One dataflow launch per sweep of every smoothed level with explicit
    patches: two per level and V-cycle."""
    from paper_2608_14310_amd import Solver
    s = workloads.beam_fibres(128, 5, 1e-2, 1e4, seed=0)
    g = Solver(0)
    try:
        g.setup(s, alpha=1.0, smoother="multiplicative")
        st = g.build_cav_patches("cav")
        g.factor_patches("fp64")
        g.set_smoother("multiplicative", 1.0)
        g.set_tuning(_table(s.n_levels, 2))
        lv = sum(1 for x in st[1:] if x["n_explicit"] > 0)
        g.kernel_timing(True)
        for _ in range(5):
            g.vcycle(_t(s.b))
        kt = g.kernel_timing(False)
        print(f"[flow] timing {kt}", flush=True)
        assert kt["flow_launches"] == 5 * 2 * lv
        assert kt["flow_bytes"] > 0 and kt["flow_ms"] > 0
    finally:
        g.close()
