"""Benchmark: CAV-multigrid FGMRES time-to-1e-10 at 512^2 (beam law, 5 levels).

One step = the whole path on the 512^2 open-fibre beam system (4 fibres of
length 0.4, ds = h/2, bending kappa_b = 1e-2, springs 1e4, 5-level V(1,1)):
build_operator -> build_cav_patches -> factor_patches -> fgmres_solve to 1e-10.
The stiffer members of the kappa_b sweep (1, 1e2) are run once after the
timed steps and reported with their iteration counts (they do not reach
1e-10 within 150 iterations at this resolution).
Inputs (markers, RHS on the device) are prepared before the timed region.
`value` is the mean wall time per solve (ms, lower is better), hierarchy
build included. The dominant kernel (explicit-patch GEMV of the smoother) is
timed live with HIP events around each of its launches on the library stream.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def measured_traffic(kernel: str, precision: str, smoother: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    passes (FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by what the
    counter reads for a plain copy of known size), or None when no pass
    covers this configuration or the kernel's source has changed since."""
    import hashlib
    try:
        with open(os.path.join(ROOT, "profiles", "counters.json")) as f:
            rec = json.load(f).get(kernel)
    except (OSError, ValueError):
        return None
    if not rec or rec["precision"] != precision or rec["smoother"] != smoother:
        return None
    with open(os.path.join(ROOT, rec["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != rec["sha256"]:
            return None
    kib = rec["fetch_kib_per_dispatch"] * rec["fetch_factor"] + rec["write_kib_per_dispatch"] * rec["write_factor"]
    return int(kib * 1024)


def cpu_baseline(kappa_b: float, iters_gpu: int, smoother: str, alpha: float, sample_patches: int = 400):
    """The FP64 oracle on a bounded sample of the same 512^2 workload, timed on
    one host core: E_E, the Galerkin hierarchy and every level's patch family
    are built in full; the local factorisations and the smoother's per-patch
    work are timed on a sample of patches per level and scaled to the level's
    patch count; one V(1,1) cycle is then two sweeps per smoothed level, and the
    solve is the GPU's iteration count of V-cycle + operator apply."""
    import numpy as np
    import scipy.sparse as sp
    from threadpoolctl import threadpool_limits

    import workloads
    from oracle import hierarchy, ib, mac, patches as pmod, smoothers

    with threadpool_limits(limits=1):
        s = workloads.beam_512(kappa_b)
        t0 = time.perf_counter()
        EE, pat = ib.eulerian_elasticity(s)
        levels = [(s.N, EE, pat)]
        for _ in range(s.n_levels - 1):
            N = levels[-1][0] // 2
            levels.append((N,) + hierarchy.galerkin(levels[-1][1], levels[-1][2], N))
        t_build = time.perf_counter() - t0
        t_fact = t_sweep = t_pat = 0.0
        rng = np.random.default_rng(0)
        for (N, E, P) in levels[:-1]:
            tp = time.perf_counter()
            ps, std = pmod.cav_patches(N, P)
            t_pat += time.perf_counter() - tp
            K = mac.reduced_operator(N, s.rho, s.mu, s.dt, E)
            Kc = K.tocsc()
            pick = rng.choice(len(ps), size=min(sample_patches, len(ps)), replace=False)
            sub = [ps[k] for k in pick]
            tf = time.perf_counter()
            sol = smoothers.PatchSolvers(K, sub, std[pick])
            t_fact += (time.perf_counter() - tf) * len(ps) / len(sub)
            r = rng.standard_normal(K.shape[0])
            ts = time.perf_counter()
            for k, p in enumerate(sub):                    # one multiplicative step per patch
                d = sol.solve_one(k, r[p])
                r -= Kc[:, p] @ d
            t_sweep += (time.perf_counter() - ts) * len(ps) / len(sub)
        K = mac.reduced_operator(s.N, s.rho, s.mu, s.dt, EE)
        ta = time.perf_counter()
        for _ in range(3):
            K @ s.b
        t_apply = (time.perf_counter() - ta) / 3
    setup = t_build + t_pat + t_fact
    per_it = 2 * t_sweep + t_apply
    total_ms = 1e3 * (setup + iters_gpu * per_it)
    return {"value": round(total_ms, 1), "unit": "ms", "cores": 1, "kind": "oracle",
            "sample": (f"512^2 beam kappa_b={kappa_b:g}, {smoother} CAV: E_E + hierarchy + patch families in full "
                       f"({t_build + t_pat:.1f} s); factorisation and one smoother step timed on {sample_patches} "
                       f"random patches per level and scaled to each level's patch count; V-cycle = 2 sweeps "
                       f"({2 * t_sweep:.1f} s est.) + K apply; extrapolated to {iters_gpu} iterations")}


def copy_calibration(nbytes: int):
    """A plain device-to-device copy of known size, for scaling HBM counters."""
    import torch
    n = nbytes // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 5}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--smoother", default="multiplicative", choices=["multiplicative", "additive"])
    ap.add_argument("--kappa-b", type=float, nargs="*", default=[1e-2])
    ap.add_argument("--stiff-sweep", type=float, nargs="*", default=[1.0, 1e2])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, help="run only a plain copy of this many bytes")
    a = ap.parse_args()
    if a.calibrate_copy:
        copy_calibration(a.calibrate_copy)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus above 1 is not supported"}))
        sys.exit(2)

    import numpy as np
    import torch

    import workloads
    from paper_2608_14310_amd import Solver

    dev = torch.device("cuda", 0)
    systems = [workloads.beam_512(kb) for kb in a.kappa_b]
    rhs = [torch.from_numpy(s.b).to(dev) for s in systems]
    g = Solver(0)
    stream = torch.cuda.current_stream(dev)
    alpha = 1.0 if a.smoother == "multiplicative" else 0.7

    def one_step(record):
        out = []
        for s, b in zip(systems, rhs):
            t0 = time.perf_counter()
            g.build_operator(s)
            t1 = time.perf_counter()
            stats = g.build_cav_patches("cav")
            t2 = time.perf_counter()
            fst = g.factor_patches(a.precision, 1e6)
            g.set_smoother(a.smoother, alpha)
            t3 = time.perf_counter()
            g.kernel_timing(True)
            x, info = g.fgmres_solve(b, rtol=1e-10, max_it=150)
            kt = g.kernel_timing(False)
            t4 = time.perf_counter()
            out.append(dict(kb=s.kappa["kappa_b"], build=t1 - t0, patches=t2 - t1, factor=t3 - t2, solve=t4 - t3,
                            its=info["iterations"], conv=info["converged"], est=info["est_rel_residual"],
                            true=info["true_rel_residual"], stats=stats, fst=fst, kt=kt))
        return out

    for _ in range(a.warmup):
        one_step(False)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    t0 = time.perf_counter()
    runs = []
    for _ in range(a.steps):
        runs.append(one_step(True))
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n_solves = a.steps * len(systems)
    ms_per_step = 1e3 * wall / a.steps
    ms_per_solve = 1e3 * wall / n_solves

    # dominant kernel: explicit-patch GEMV, bytes and time accumulated by the library
    kb_bytes = sum(r["kt"]["bytes"] for run in runs for r in run)
    kb_ms = sum(r["kt"]["ms"] for run in runs for r in run)
    kb_launch = sum(r["kt"]["launches"] for run in runs for r in run)
    achieved = kb_bytes / (kb_ms * 1e-3) / 1e9 if kb_ms > 0 else 0.0
    last = runs[-1]
    per_sys = [{k: (float("%.4g" % v) if isinstance(v, float) else v) for k, v in r.items()
                if k not in ("stats", "fst", "kt")} for r in last]
    vcycle_ms = [r["kt"]["vcycle_ms"] for r in last]
    line = {
        "metric": "FGMRES(CAV-MG) time-to-1e-10 rel. residual at 512^2; V-cycle HBM GB/s",
        "value": round(ms_per_solve, 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if a.precision == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {"workload": "beam512: 512x512 MAC grid, 5-level V(1,1), 4 open fibres L=0.4 ds=h/2, "
                               "kappa_b sweep " + ",".join(f"{k:g}" for k in a.kappa_b) +
                               ", kappa_s=1e4, rho=1 mu=0.01 dt=1e-3, seeded U[-1,1] RHS, FGMRES rtol 1e-10",
                   "precision": a.precision, "smoother": a.smoother, "alpha": alpha},
        "per_system": per_sys,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic("k_mult_exp" if a.smoother == "multiplicative" else "k_patch_apply",
                                                 a.precision, a.smoother),
                     "kernel": "k_mult_exp" if a.smoother == "multiplicative" else "k_patch_apply",
                     "launches": kb_launch,
                     "bytes_per_launch": int(kb_bytes / max(kb_launch, 1)),
                     "avg_launch_us": round(1e3 * kb_ms / max(kb_launch, 1), 3)},
        "vcycle_ms": [round(v, 4) for v in vcycle_ms],
    }
    sweep = []
    for kb in a.stiff_sweep:
        s = workloads.beam_512(kb)
        g.build_operator(s)
        g.build_cav_patches("cav")
        g.factor_patches(a.precision, 1e6)
        g.set_smoother(a.smoother, alpha)
        t0s = time.perf_counter()
        _, inf = g.fgmres_solve(torch.from_numpy(s.b).to(dev), rtol=1e-10, max_it=150)
        torch.cuda.synchronize()
        sweep.append({"kappa_b": kb, "iterations": inf["iterations"], "converged": inf["converged"],
                      "est_rel_residual": inf["est_rel_residual"], "solve_ms": round(1e3 * (time.perf_counter() - t0s), 1)})
    line["stiffness_sweep"] = sweep
    if a.verbose:
        line["level_stats"] = last[0]["stats"]
        line["factor_stats"] = [r["fst"] for r in last]
    if not a.no_cpu_baseline:
        mid = last[len(last) // 2]
        line["cpu_baseline"] = cpu_baseline(mid["kb"], mid["its"], a.smoother, alpha)
    g.close()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
