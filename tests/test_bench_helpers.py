"""Host logic of the benchmark's accounting (no GPU): the algorithmic bytes of
a V(k,k) cycle, the choice of the dominant kernel from live timing brackets,
and the reduction of rocprofv3 counter CSVs."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def _stats():
    # level 0 (coarsest) carries no patches; levels 1.. are smoothed
    return [None,
            {"avg_np": 6.0, "n_patches": 64 * 64, "n_explicit": 100, "ee_nnz": 5000},
            {"avg_np": 7.0, "n_patches": 128 * 128, "n_explicit": 300, "ee_nnz": 20000}]


def test_vcycle_bytes_counts_each_sweep_once():
    st, fst = _stats(), {"factor_bytes": 1.0e8}
    N, L = 128, 3
    one = bench.vcycle_bytes(st, fst, N, L, "fp64")
    # by hand for V(1,1): two sweeps per smoothed level, then the coarsest inverse
    ref = 0.0
    for lvl in (1, 2):
        s = st[lvl]
        nl = N >> (L - 1 - lvl)
        sum_np = s["avg_np"] * s["n_patches"] - 5.0 * (s["n_patches"] - s["n_explicit"])
        ref += 2 * 20.0 * sum_np + 10 * 3 * nl * nl * 8.0 + 2 * s["ee_nnz"] * 12.0
    ref += 2 * fst["factor_bytes"] + (3 * (N >> (L - 1)) ** 2) ** 2 * 8.0
    assert one == pytest.approx(ref, rel=1e-12)
    # V(3,3): every per-sweep term three times, the coarsest solve once
    three = bench.vcycle_bytes(st, fst, N, L, "fp64", sweeps=3)
    coarse = (3 * (N >> (L - 1)) ** 2) ** 2 * 8.0
    assert three - coarse == pytest.approx(3 * (one - coarse), rel=1e-12)


def _kt(ms=0.0, coop_ms=0.0, shared_ms=0.0, flow_ms=0.0, launches=10):
    return {"ms": ms, "bytes": 100.0 * launches, "launches": launches,
            "coop_ms": coop_ms, "coop_bytes": 40.0 * launches if coop_ms else 0.0,
            "coop_launches": launches // 2 if coop_ms else 0,
            "shared_ms": shared_ms, "shared_bytes": 30.0 * launches if shared_ms else 0.0,
            "shared_launches": launches // 2 if shared_ms else 0,
            "flow_ms": flow_ms, "flow_bytes": 20.0 * launches if flow_ms else 0.0,
            "flow_launches": 1 if flow_ms else 0}


def test_dominant_kernel_follows_the_larger_bracket_time():
    # additive: no cooperative or flow brackets, every byte is k_add_smooth's
    name, b, ms, n = bench.dominant_kernel([_kt(ms=5.0)], "additive", "default")
    assert (name, b, ms, n) == ("k_add_smooth", 1000.0, 5.0, 10)
    # multiplicative with the shared-residual form holding most of the time
    name, b, ms, n = bench.dominant_kernel([_kt(ms=10.0, coop_ms=8.0, shared_ms=7.0)], "multiplicative", "default")
    assert (name, b, ms, n) == ("k_mult_coopr", 300.0, 7.0, 5)
    # the dataflow sweep when its brackets dominate
    name, _, ms, _ = bench.dominant_kernel([_kt(ms=10.0, flow_ms=9.0)], "multiplicative", "default")
    assert (name, ms) == ("k_mult_flow", 9.0)
    # several steps add up
    name, b, ms, n = bench.dominant_kernel([_kt(ms=5.0), _kt(ms=3.0)], "additive", "default")
    assert (b, ms, n) == (2000.0, 8.0, 20)


def test_summarize_counters_averages_per_kernel_and_counter(tmp_path):
    p = tmp_path / "c.csv"
    p.write_text("Kernel_Name,Counter_Name,Counter_Value\n"
                 "\"void cav::(anonymous namespace)::k_add_smooth<true>(int, double)\",FETCH_SIZE,10\n"
                 "\"void cav::(anonymous namespace)::k_add_smooth<true>(int, double)\",FETCH_SIZE,30\n"
                 "\"cav::(anonymous namespace)::k_touched(int)\",FETCH_SIZE,4\n")
    out = bench.summarize_counters(str(p))
    assert out["k_add_smooth<true>"]["FETCH_SIZE"] == {"dispatches": 2, "mean": 20.0}
    assert out["k_touched"]["FETCH_SIZE"] == {"dispatches": 1, "mean": 4.0}
