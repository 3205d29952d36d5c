"""Benchmark: CAV-multigrid FGMRES time-to-1e-10 at 512^2 (beam law, 5 levels).

One step = the whole path on the 512^2 open-fibre beam system (4 fibres of
length 0.4, ds = h/2, bending kappa_b = 1e-2, springs 1e4, 5-level V(1,1)):
build_operator -> build_cav_patches -> factor_patches -> fgmres_solve to 1e-10.
`value` is the mean wall time per step (T_total, ms, lower is better);
`t_solve_ms` is the solve alone. Inputs (markers, RHS on the device) are
prepared before the timed region; the smoother follows the library's
default table (a launch per colour phase in the cooperative form with a
shared residual; the autotuned table, which may pick the one-launch dataflow
sweep per level, is measured and reported after the timed steps).
The dominant kernel (the explicit-patch kernel of the multiplicative
smoother) is timed live with HIP events on the library stream around its
launches.
After the timed steps: the other precision on the same system, the stiffer
kappa_b values (reported with their iteration counts), the weighted additive
smoother (its V-cycle here, time-to-1e-10 on the 256^2 membrane), the
learned stage (trained on 256^2 pairs, judged on this solve), the batched
mix of independent systems in one captured graph, and the CPU oracle (a
bounded sample of this workload, and whole solves of the 32^2 and 256^2
systems). `vcycle_gbs` is the V-cycle's algorithmic bytes over its time.
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


def measured_traffic(kernel: str, precision: str, smoother: str, tune: str, layout: str = "full"):
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
    if (not rec or rec["precision"] != precision or rec["smoother"] != smoother or rec.get("tune", "default") != tune
            or rec.get("layout", "full") != layout):
        return None
    with open(os.path.join(ROOT, rec["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != rec["sha256"]:
            return None
    kib = rec["fetch_kib_per_dispatch"] * rec["fetch_factor"] + rec["write_kib_per_dispatch"] * rec["write_factor"]
    return int(kib * 1024)


def host_cores() -> int:
    """Host cores this process may use (its affinity set, capped by OMP_NUM_THREADS)."""
    n = len(os.sched_getaffinity(0))
    try:
        n = min(n, int(os.environ.get("OMP_NUM_THREADS", n)))
    except ValueError:
        pass
    return max(n, 1)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_sampled_512(kappa_b: float, iters_gpu: int, threads: int, sample_patches: int, sweeps: int = 1):
    """The FP64 oracle's multiplicative cycle on a bounded sample of the 512^2
    headline workload with `threads` BLAS threads: E_E, the Galerkin hierarchy
    and every level's patch family are built in full; the local
    factorisations and the multiplicative smoother's per-patch work (local
    solve and residual update, one patch at a time as the oracle's sweep does
    it) are timed on a sample of patches per level and scaled to the level's
    patch count; one V(sweeps, sweeps) cycle is then 2 sweeps sweeps per
    smoothed level, and the solve is the GPU's iteration count of V-cycle +
    operator apply. Returns (total ms, sweep s, build s)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import workloads
    from oracle import hierarchy, ib, mac, patches as pmod, smoothers

    with threadpool_limits(limits=threads):
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
    per_it = 2 * sweeps * t_sweep + t_apply
    return 1e3 * (setup + iters_gpu * per_it), 2 * sweeps * t_sweep, t_build + t_pat


def cpu_additive_512(kappa_b: float, iters_gpu: int, threads: int, alpha: float, sweeps: int):
    """The FP64 oracle's weighted additive cycle on the 512^2 headline
    workload: the whole hierarchy (E_E, Galerkin levels, patch families, every
    local LU factorisation) built with `threads` BLAS threads, one whole
    V(sweeps, sweeps) cycle and one operator apply timed with all of them and
    again with one thread, each extrapolated to the GPU's iteration count.
    Returns (total ms, total ms on one thread, setup s, cycle s, cycle s on
    one thread)."""
    from threadpoolctl import threadpool_limits

    import workloads
    from oracle import multigrid
    s = workloads.beam_512(kappa_b)
    with threadpool_limits(limits=threads):
        t0 = time.perf_counter()
        H = multigrid.Hierarchy(s, alpha=alpha, smoother="additive", pre=sweeps, post=sweeps)
        K = H.levels[-1].K
        t_setup = time.perf_counter() - t0
        t1 = time.perf_counter()
        H.vcycle(s.b)
        K @ s.b
        t_cycle = time.perf_counter() - t1
    with threadpool_limits(limits=1):
        t2 = time.perf_counter()
        H.vcycle(s.b)
        K @ s.b
        t_cycle1 = time.perf_counter() - t2
    return (1e3 * (t_setup + iters_gpu * t_cycle), 1e3 * (t_setup + iters_gpu * t_cycle1), t_setup, t_cycle,
            t_cycle1)


def cpu_full_solve(system, alpha: float, threads: int):
    """A whole oracle FGMRES solve (setup, then the solve to 1e-10) with the
    weighted additive CAV V(1,1) cycle and `threads` BLAS threads."""
    from threadpoolctl import threadpool_limits

    from oracle import krylov, multigrid
    with threadpool_limits(limits=threads):
        t0 = time.perf_counter()
        H = multigrid.Hierarchy(system, alpha=alpha, smoother="additive")
        K = H.levels[-1].K
        t1 = time.perf_counter()
        res = krylov.fgmres(lambda v: K @ v, H.vcycle, system.b, 1e-10, 150)
        t2 = time.perf_counter()
    return {"setup_ms": round(1e3 * (t1 - t0), 1), "solve_ms": round(1e3 * (t2 - t1), 1),
            "total_ms": round(1e3 * (t2 - t0), 1), "iterations": res.iterations, "threads": threads}


def cpu_baseline(kappa_b: float, iters_gpu: int, smoother: str, gpu_full: dict, sample_patches: int = 200,
                 alpha: float = 1.0, sweeps: int = 1):
    """The oracle as it stands, on the host cores: the headline workload on a
    bounded sample (extrapolated, all host cores and 1 thread), and whole
    solves of the 32^2 target and 256^2 membrane systems (additive cycle,
    all host cores and 1 thread) beside the GPU's solves of the same systems
    in this run."""
    import workloads
    cores = host_cores()
    if smoother == "additive":
        total, total1, t_setup, t_cyc, t_cyc1 = cpu_additive_512(kappa_b, iters_gpu, cores, alpha, sweeps)
        sample = (f"512^2 beam kappa_b={kappa_b:g}, weighted additive CAV V({sweeps},{sweeps}) alpha {alpha:g}: "
                  f"the oracle's hierarchy built in full with {cores} BLAS threads ({t_setup:.1f} s), one whole "
                  f"V-cycle + K apply timed with {cores} threads ({t_cyc:.1f} s) and with 1 thread "
                  f"({t_cyc1:.1f} s, setup taken from the all-core run), extrapolated to {iters_gpu} iterations "
                  "(an extrapolation, not a whole solve)")
    else:
        total, sweep_s, build_s = cpu_sampled_512(kappa_b, iters_gpu, cores, sample_patches, sweeps)
        total1, _, _ = cpu_sampled_512(kappa_b, iters_gpu, 1, sample_patches, sweeps)
        sample = (f"512^2 beam kappa_b={kappa_b:g}, multiplicative CAV V({sweeps},{sweeps}), "
                  f"{cores} BLAS threads: E_E + hierarchy + "
                  f"patch families in full ({build_s:.1f} s); factorisation and one smoother step timed on "
                  f"{sample_patches} random patches per level and scaled to each level's patch count; "
                  f"V-cycle = {2 * sweeps} sweeps ({sweep_s:.1f} s est.) + K apply; extrapolated to "
                  f"{iters_gpu} iterations (an extrapolation, not a whole solve)")
    full = {}
    for key, system in (("target32", workloads.small_target(0)), ("membrane256", workloads.membrane_256(1e4))):
        rows = [cpu_full_solve(system, 0.7, t) for t in (cores, 1)]
        full[key] = {"all_cores": rows[0], "one_thread": rows[1], "gpu": gpu_full.get(key)}
    return {"value": round(total, 1), "unit": "ms", "cores": cores, "kind": "oracle",
            "sample": sample,
            "one_thread_value": round(total1, 1), "cpu_model": cpu_model(),
            "threads": {"blas": cores, "python": 1},
            "full_solves": full}


def vcycle_bytes(stats, fst, N: int, n_levels: int, precision: str, sweeps: int = 1) -> float:
    """Algorithmic HBM bytes of one V(sweeps, sweeps) cycle (what the method
    must move): per smoothed level 2 * sweeps sweeps, each streaming its
    explicit patches' inverses (sum n_p^2 s; the shared far-field inverse is
    free) and their index / gathered residual / update (20 B per patch
    unknown), about five vector passes per sweep (residual, transfers, mean
    removal, far-field colours) and the E_E rows of one operator apply per
    sweep (12 B per nonzero); then the dense coarsest solution operator once
    (n_c^2 8 B)."""
    total = 0.0
    fbytes = float(fst["factor_bytes"])  # per sweep, all levels, at the stored precisions
    k = 2 * sweeps
    for l in range(1, n_levels):
        st = stats[l]
        Nl = N >> (n_levels - 1 - l)
        sum_np = st["avg_np"] * st["n_patches"] - 5.0 * (st["n_patches"] - st["n_explicit"])
        total += k * 20.0 * sum_np + 5 * k * 3 * Nl * Nl * 8.0 + k * st["ee_nnz"] * 12.0
    total += k * fbytes
    nc = 3 * (N >> (n_levels - 1)) ** 2
    return total + nc * nc * 8.0


# storage of the patch inverses for the additive smoother: the symmetric
# panel layout (lower panels only) unless --layout full; the multiplicative
# kernels always get the full layout
ADD_LAYOUT = "symmetric"


def _layout(smoother: str) -> str:
    return ADD_LAYOUT if smoother == "additive" else "full"


def additive_leg(dev, reps: int = 10, membrane: bool = True):
    """North-star smoother (Appendix A, weighted additive CAV, alpha 0.7): its
    V-cycle on the 512^2 beam system (FGMRES with it stalls there, so only
    the cycle is timed), with the patch-inverse GEMV kernel's live
    bandwidth; then time-to-1e-10 on the 256^2 membrane (kappa_s = 1e4),
    where it converges, beside the multiplicative cycle."""
    import torch

    import workloads
    from paper_2608_14310_amd import Solver
    s = workloads.beam_512(1e-2)
    g = Solver(0)
    stats, fst = g.setup(s, precision="fp64", alpha=0.7, smoother="additive", layout=_layout("additive"))
    b = torch.from_numpy(s.b).to(dev)
    for _ in range(2):
        g.vcycle(b)
    torch.cuda.synchronize()
    g.kernel_timing(True)
    for _ in range(reps):
        g.vcycle(b)
    kt = g.kernel_timing(False)
    g.close()
    bv = vcycle_bytes(stats, fst, s.N, s.n_levels, "fp64")
    pa_ms = kt["ms"] - kt["coop_ms"] - kt["flow_ms"]
    pa_bytes = kt["bytes"] - kt["coop_bytes"] - kt["flow_bytes"]
    pa_launch = kt["launches"] - kt["coop_launches"] - kt["flow_launches"]
    pa_gbs = pa_bytes / (pa_ms * 1e-3) / 1e9 if pa_ms > 0 else 0.0
    out = {"workload": "beam512 (as the headline), weighted additive CAV V(1,1), alpha 0.7, FP64 factors, "
                       f"{_layout('additive')} layout",
           "vcycle_ms": round(kt["vcycle_ms"], 4), "vcycles_per_s": round(1e3 / kt["vcycle_ms"], 1),
           "vcycle_bytes": int(bv), "vcycle_gbs": round(bv / (kt["vcycle_ms"] * 1e-3) / 1e9, 1),
           "vcycle_frac": round(bv / (kt["vcycle_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "k_add_smooth": {"bound": "hbm", "achieved": round(pa_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(pa_gbs / HBM_PEAK_GBS, 4),
                             "traffic": measured_traffic("k_add_smooth", "fp64", "additive", "default",
                                                         _layout("additive")),
                             "launches": pa_launch,
                             "bytes_per_launch": int(pa_bytes / max(pa_launch, 1)),
                             "avg_launch_us": round(1e3 * pa_ms / max(pa_launch, 1), 3)}}
    if not membrane:
        return out
    # time-to-1e-10 where the additive cycle converges
    sm = workloads.membrane_256(1e4)
    bm = torch.from_numpy(sm.b).to(dev)
    rows = {}
    for smoother, alpha in (("additive", 0.7), ("multiplicative", 1.0)):
        g = Solver(0)
        g.setup(sm, precision="fp64", alpha=alpha, smoother=smoother, layout=_layout(smoother))
        g.fgmres_solve(bm, rtol=1e-10, max_it=150)     # warm-up
        times = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.build_operator(sm)
            g.build_cav_patches("cav")
            g.factor_patches("fp64", 1e6)
            g.set_smoother(smoother, alpha)
            t1 = time.perf_counter()
            _, inf = g.fgmres_solve(bm, rtol=1e-10, max_it=150)
            torch.cuda.synchronize()
            times.append((t1 - t0, time.perf_counter() - t1))
        g.close()
        ts = sorted(times, key=lambda v: v[0] + v[1])[1]
        rows[smoother] = {"iterations": inf["iterations"], "converged": inf["converged"],
                          "true_rel_residual": float("%.3g" % inf["true_rel_residual"]),
                          "t_total_ms": round(1e3 * (ts[0] + ts[1]), 2), "t_solve_ms": round(1e3 * ts[1], 2)}
    out["membrane256"] = dict(workload="membrane256: 256x256, ellipse 0.2/0.15, kappa_s=1e4, 6 levels, FP64",
                              **rows)
    return out


def additive_sweeps_leg(dev, alpha: float = 0.9, sweeps: int = 3):
    """The weighted additive CAV cycle with more smoothing (damping alpha,
    V(sweeps, sweeps)) on the headline system, FP64 and FP32 factors, as a
    whole timed step (operator, patches, factors, solve) beside the paper's
    V(1,1) multiplicative headline; the FP64 path's iteration count is
    pinned to the oracle's golden for this configuration."""
    import torch

    import workloads
    from paper_2608_14310_amd import Solver
    s = workloads.beam_512(1e-2)
    b = torch.from_numpy(s.b).to(dev)
    g = Solver(0)
    out = {"workload": f"beam512 (as the headline), weighted additive CAV, alpha {alpha:g}, V({sweeps},{sweeps}), "
                       f"{_layout('additive')} layout"}
    xs = {}
    for prec in ("fp64", "mixed"):
        stats, fst = g.setup(s, precision=prec, alpha=alpha, smoother="additive", layout=_layout("additive"))
        g.set_smoother("additive", alpha, sweeps, sweeps)
        g.fgmres_solve(b, rtol=1e-10, max_it=150)      # warm-up
        best = None
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.build_operator(s)
            g.build_cav_patches("cav")
            fst = g.factor_patches(prec, 1e6)
            g.set_smoother("additive", alpha, sweeps, sweeps)
            t1 = time.perf_counter()
            g.kernel_timing(True)
            x, inf = g.fgmres_solve(b, rtol=1e-10, max_it=150)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            kt = g.kernel_timing(False)
            if best is None or t2 - t0 < best[0]:
                best = (t2 - t0, t2 - t1, inf, kt, x)
        tt, ts, inf, kt, x = best
        xs[prec] = x
        bv = vcycle_bytes(stats, fst, s.N, s.n_levels, prec, sweeps)
        out[prec] = {"iterations": inf["iterations"], "converged": inf["converged"],
                     "true_rel_residual": float("%.3g" % inf["true_rel_residual"]),
                     "t_total_ms": round(1e3 * tt, 2), "t_solve_ms": round(1e3 * ts, 2),
                     "vcycle_ms": round(kt["vcycle_ms"], 4), "vcycle_bytes": int(bv),
                     "vcycle_gbs": round(bv / (kt["vcycle_ms"] * 1e-3) / 1e9, 1),
                     "vcycle_frac": round(bv / (kt["vcycle_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    out["mixed"]["rel_err_vs_fp64"] = float(
        "%.3g" % (torch.linalg.norm(xs["mixed"] - xs["fp64"]) / torch.linalg.norm(xs["fp64"])).item())
    g.close()
    return out


def dominant_kernel(kts, smoother: str, tune: str):
    """The dominant smoothing kernel of timed solves from their live HIP-event
    brackets (cav_kernel_timing): the dataflow sweep when its brackets hold
    most of the time, else the shared-residual form, else the other
    cooperative forms, else the one-workgroup phase form (multiplicative) or
    k_add_smooth (additive). Returns (name, bytes, ms, launches)."""
    co_ms = sum(k["coop_ms"] for k in kts)
    sh_ms = sum(k["shared_ms"] for k in kts)
    fl_ms = sum(k["flow_ms"] for k in kts)
    all_ms = sum(k["ms"] for k in kts)
    if fl_ms > all_ms - fl_ms:
        return ("k_mult_flow", sum(k["flow_bytes"] for k in kts), fl_ms, sum(k["flow_launches"] for k in kts))
    if sh_ms > all_ms - sh_ms:
        return ("k_mult_coopr", sum(k["shared_bytes"] for k in kts), sh_ms,
                sum(k["shared_launches"] for k in kts))
    if co_ms > all_ms - co_ms:
        name = {"coop64": "k_mult_coop<64>", "coop128": "k_mult_coop<128>"}.get(tune, "k_mult_coop")
        return (name, sum(k["coop_bytes"] - k["shared_bytes"] for k in kts), co_ms - sh_ms,
                sum(k["coop_launches"] - k["shared_launches"] for k in kts))
    name = "k_mult_exp" if smoother == "multiplicative" else "k_add_smooth"
    return (name, sum(k["bytes"] - k["coop_bytes"] - k["flow_bytes"] for k in kts), all_ms - co_ms - fl_ms,
            sum(k["launches"] - k["coop_launches"] - k["flow_launches"] for k in kts))


def paper_v11_leg(dev, kappa_b: float, steps: int = 2):
    """The paper's cycle on the headline system: coloured multiplicative CAV
    V(1,1) (standard-first phase order), FP64 factors, whole timed steps
    (operator, patches, factors, solve) after one untimed one, with the
    dominant phase kernel's live bandwidth and its counter-derived traffic;
    then the same with FP32 factors. Its FP64 iteration count is pinned to
    the oracle's golden."""
    import torch

    import workloads
    from paper_2608_14310_amd import Solver
    s = workloads.beam_512(kappa_b)
    b = torch.from_numpy(s.b).to(dev)
    g = Solver(0)

    def step(prec):
        t0 = time.perf_counter()
        g.build_operator(s)
        stats = g.build_cav_patches("cav")
        fst = g.factor_patches(prec, 1e6)
        g.set_smoother("multiplicative", 1.0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g.kernel_timing(True)
        x, inf = g.fgmres_solve(b, rtol=1e-10, max_it=150)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return dict(total=t2 - t0, solve=t2 - t1, inf=inf, kt=g.kernel_timing(False), stats=stats, fst=fst, x=x)

    step("fp64")
    runs = [step("fp64") for _ in range(steps)]
    kernel, kb_bytes, kb_ms, kb_launch = dominant_kernel([r["kt"] for r in runs], "multiplicative", "default")
    achieved = kb_bytes / (kb_ms * 1e-3) / 1e9 if kb_ms > 0 else 0.0
    last = runs[-1]
    bv = vcycle_bytes(last["stats"], last["fst"], s.N, s.n_levels, "fp64", 1)
    vc = last["kt"]["vcycle_ms"]
    mixed = step("mixed")
    out = {"workload": "beam512 (as the headline), coloured multiplicative CAV V(1,1), alpha 1, standard-first "
                       "phase order: the paper's cycle",
           "t_total_ms": round(1e3 * min(r["total"] for r in runs), 2),
           "t_solve_ms": round(1e3 * min(r["solve"] for r in runs), 2),
           "iterations": last["inf"]["iterations"], "converged": last["inf"]["converged"],
           "true_rel_residual": float("%.3g" % last["inf"]["true_rel_residual"]),
           "vcycle_ms": round(vc, 4), "vcycle_bytes": int(bv), "vcycle_gbs": round(bv / (vc * 1e-3) / 1e9, 1),
           "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4),
                        "traffic": measured_traffic(kernel, "fp64", "multiplicative", "default"),
                        "kernel": kernel, "launches": kb_launch, "bytes_per_launch": int(kb_bytes / max(kb_launch, 1)),
                        "avg_launch_us": round(1e3 * kb_ms / max(kb_launch, 1), 3)},
           "mixed": {"t_total_ms": round(1e3 * mixed["total"], 2), "t_solve_ms": round(1e3 * mixed["solve"], 2),
                     "iterations": mixed["inf"]["iterations"],
                     "true_rel_residual": float("%.3g" % mixed["inf"]["true_rel_residual"]),
                     "rel_err_vs_fp64": float("%.3g" % (torch.linalg.norm(mixed["x"] - last["x"]) /
                                                        torch.linalg.norm(last["x"])).item())}}
    g.close()
    return out


def membrane_leg(dev, kappas=(1e2, 1e4, 1e6)):
    """The 256^2 membrane (ellipse 0.2/0.15, nearest-neighbour springs,
    ds = h/2) at each stiffness, FGMRES to 1e-10, with the headline cycle
    (weighted additive, alpha 0.9, V(3,3)) and the paper's multiplicative
    V(1,1): FP64 factors against FP32 factors with FP64 FGMRES, and each mixed
    solution's error against the FP64 one (the FP64 paths are pinned to the
    oracle's goldens for these systems)."""
    import torch

    import workloads
    from paper_2608_14310_amd import Solver
    out = []
    for ks in kappas:
        sm = workloads.membrane_256(ks)
        bm = torch.from_numpy(sm.b).to(dev)
        g = Solver(0)
        row = {"kappa_s": ks}
        for key, smoother, alpha, sweeps in (("additive_v33", "additive", 0.9, 3),
                                              ("multiplicative_v11", "multiplicative", 1.0, 1)):
            xs = {}
            row[key] = {}
            for prec in ("fp64", "mixed"):
                g.setup(sm, precision=prec, alpha=alpha, smoother=smoother, layout=_layout(smoother))
                g.set_smoother(smoother, alpha, sweeps, sweeps)
                g.fgmres_solve(bm, rtol=1e-10, max_it=150)      # warm-up
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                g.build_operator(sm)
                g.build_cav_patches("cav")
                fst = g.factor_patches(prec, 1e6)
                g.set_smoother(smoother, alpha, sweeps, sweeps)
                t1 = time.perf_counter()
                x, inf = g.fgmres_solve(bm, rtol=1e-10, max_it=150)
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                xs[prec] = x
                row[key][prec] = {"iterations": inf["iterations"], "converged": inf["converged"],
                                  "status": inf.get("status", 0),
                                  "true_rel_residual": float("%.3g" % inf["true_rel_residual"]),
                                  "t_total_ms": round(1e3 * (t2 - t0), 2), "t_solve_ms": round(1e3 * (t2 - t1), 2),
                                  "n_fp32_patches": fst["n_fp32"], "n_fp64_patches": fst["n_fp64"]}
            row[key]["mixed"]["rel_err_vs_fp64"] = float(
                "%.3g" % (torch.linalg.norm(xs["mixed"] - xs["fp64"]) / torch.linalg.norm(xs["fp64"])).item())
        g.close()
        out.append(row)
    return {"workload": "membrane256: 256x256, ellipse 0.2/0.15, 6 levels, FGMRES rtol 1e-10", "runs": out}

def measure_read(nbytes: int) -> dict:
    """A plain streaming read of known size (torch's sum over float64), timed
    with events: the read rate HBM sustains on this part, for comparing a
    kernel's achieved bandwidth with what a pure read stream reaches."""
    import torch
    n = nbytes // 8
    x = torch.rand(n, dtype=torch.float64, device="cuda")
    for _ in range(3):
        x.sum()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record()
    for _ in range(reps):
        x.sum()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del x
    return {"read_bytes": n * 8, "us_per_read": round(1e3 * ms, 2), "read_gbs": round(n * 8 / (ms * 1e-3) / 1e9, 1)}


def read_calibration(nbytes: int):
    print(json.dumps(measure_read(nbytes)))


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


def batched_leg(n_systems: int, max_it: int):
    """Independent systems of the batched mix (grids 64..512, target /
    membrane / beam laws, stiffness log-uniform 1e2..1e6), mixed precision,
    multiplicative CAV V-cycle, all unfinished systems advanced one FGMRES
    iteration per launch of one captured graph. Setup is outside the timing."""
    import torch

    import workloads
    from paper_2608_14310_amd import Solver, batch_solve
    systems = workloads.batched_mix(n_systems)
    solvers = []
    t0 = time.perf_counter()
    for s in systems:
        g = Solver(0)
        g.setup(s, precision="mixed", alpha=1.0, smoother="multiplicative")
        solvers.append(g)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    bs = [torch.from_numpy(s.b).to(torch.device("cuda", 0)) for s in systems]
    batch_solve(solvers, bs, 1e-10, max_it, 0)          # warm-up: captures and first replays
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, infos, st = batch_solve(solvers, bs, 1e-10, max_it, 0)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for g in solvers:
        g.close()
    its = [i["iterations"] for i in infos]
    return {"systems": n_systems, "grids": sorted({s.N for s in systems}), "seconds": round(dt, 3),
            "solves_per_s": round(n_systems / dt, 2), "vcycles_per_s": round(sum(its) / dt, 1),
            "converged": int(sum(i["converged"] for i in infos)), "iterations_min_max": [min(its), max(its)],
            "rounds": st["rounds"], "graph_launches": st["graph_launches"], "captures": st["captures"],
            "setup_s": round(t_setup, 2), "max_it": max_it, "precision": "mixed", "mode": "one graph per round"}


def learned_leg(g_eval, b_eval, train_pairs: int, steps: int):
    """Train the learned stage on V-cycle pairs of a 256^2 beam system
    (minimal-residual loss) and judge it on the 512^2 solve: kept only if it
    cuts the iteration count."""
    import numpy as np
    import torch

    import workloads
    from paper_2608_14310_amd import Net, Solver
    from paper_2608_14310_amd import learned as LN
    dev = torch.device("cuda", 0)
    st = workloads.beam_fibres(N=256, n_levels=4, kappa_b=1e-2, seed=1)
    gt = Solver(0)
    gt.setup(st, precision="mixed", alpha=1.0, smoother="multiplicative")
    t0 = time.perf_counter()
    xs = torch.from_numpy(workloads.random_solutions(st.N, max(train_pairs // 3, 1), 1)).to(dev)
    rh, eh = LN.generate_pairs(gt, xs, 3)
    net = Net(0, workloads.net_init(0, out_scale=1e-2))
    losses = LN.train(net, rh, eh, st.N, workloads.batch_order(rh.shape[0], 8, steps, 0), 1e-3, solver=gt,
                      kind="minres")
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    gt.close()
    enabled, rows = LN.validate(g_eval, net, [b_eval])
    g_eval.attach_net(None)
    net.close()
    return {"train": f"{rh.shape[0]} pairs from 256^2 beam V-cycles, {steps} Adam steps (batch 8, minimal-residual loss)",
            "train_s": round(t_train, 2), "loss_first": round(float(np.mean(losses[:20])), 4),
            "loss_last": round(float(np.mean(losses[-50:])), 4), "eval": "512^2 beam kappa_b=1e-2, rtol 1e-10",
            "plain_its": rows[0]["plain"], "learned_its": rows[0]["learned"], "accepted": rows[0]["accepted"],
            "enabled": enabled}


def learned_c5_leg(dev, pairs_per_class: int = 10000, steps: int = 2000, eval_N: int = 1024,
                   eval_precision: str = "mixed"):
    """The learned stage at its configured scale: 20k (residual, error) pairs
    from CAV V-cycles on 256^2 membrane (kappa_s = 1e4) and beam (kappa_b =
    1e-2) systems (3 pairs per exact solution), minimal-residual training on
    the GPU through each class's own K_E, then FGMRES to 1e-10 at eval_N^2
    on a membrane and a beam system, plain CAV against CAV + stage (the plain
    cycle judges every application and is the fallback). Reports iterations,
    time and accepted / rejected applications per solve."""
    import numpy as np
    import torch

    import workloads
    from paper_2608_14310_amd import Net, Solver
    from paper_2608_14310_amd import learned as LN
    classes = [("membrane", workloads.membrane_ellipse(256, None, 1e4, seed=1)),
               ("beam", workloads.beam_fibres(256, workloads.levels_to(256, 8), 1e-2, 1e4, seed=1))]
    t0 = time.perf_counter()
    data = []
    for ci, (name, st) in enumerate(classes):
        g = Solver(0)
        g.setup(st, precision="mixed", alpha=1.0, smoother="multiplicative")
        count = (pairs_per_class + 2) // 3
        rs, es = [], []
        for k in range(0, count, 64):
            xs = torch.from_numpy(workloads.random_solutions(st.N, min(64, count - k), 1000 * (ci + 1) + k // 64)).to(dev)
            r, e = LN.generate_pairs(g, xs, 3, chunk=64)
            rs.append(r)
            es.append(e)
        data.append((g, torch.cat(rs)[:pairs_per_class], torch.cat(es)[:pairs_per_class]))
    torch.cuda.synchronize()
    t_pairs = time.perf_counter() - t0
    net = Net(0, workloads.net_init(0, out_scale=1e-2))
    t0 = time.perf_counter()
    losses = []
    orders = [workloads.batch_order(pairs_per_class, 8, steps // 2, ci) for ci in range(2)]
    for k in range(steps // 2):
        for ci in range(2):
            g, rh, eh = data[ci]
            losses.append(g.train_net_residual(net, rh, next(orders[ci]), 1e-3, "minres"))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    for g, rh, eh in data:
        g.close()
    del data
    torch.cuda.empty_cache()
    L = workloads.levels_to(eval_N, 8)
    evals = []
    for name, se in (("membrane", workloads.membrane_ellipse(eval_N, L, 1e4, seed=2)),
                     ("beam", workloads.beam_fibres(eval_N, L, 1e-2, 1e4, seed=2))):
        g = Solver(0)
        g.setup(se, precision=eval_precision, alpha=1.0, smoother="multiplicative")
        b = torch.from_numpy(se.b).to(dev)
        g.attach_net(net, 1e-3)
        row = {"system": f"{name} {eval_N}^2, {L} levels, {eval_precision} factors", "unknowns": se.n}
        for mode in ("plain", "learned"):
            g.fgmres_solve(b, 1e-10, 150, learned=mode == "learned")   # warm-up
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, inf = g.fgmres_solve(b, 1e-10, 150, learned=mode == "learned")
            torch.cuda.synchronize()
            row[mode] = {"iterations": inf["iterations"], "converged": inf["converged"],
                         "true_rel_residual": float("%.3g" % inf["true_rel_residual"]),
                         "solve_ms": round(1e3 * (time.perf_counter() - t1), 1),
                         "accepted": inf["learned_accepted"], "rejected": inf["learned_rejected"]}
        g.attach_net(None)
        g.close()
        evals.append(row)
    net.close()
    return {"train": f"{2 * pairs_per_class} pairs (256^2 membrane kappa_s=1e4 and beam kappa_b=1e-2, 3 V-cycle "
                     f"iterations per exact solution), {steps} Adam steps (batch 8, minimal-residual loss through "
                     "each class's K_E)",
            "pairs_s": round(t_pairs, 2), "train_s": round(t_train, 2),
            "loss_first": round(float(np.mean(losses[:40])), 4), "loss_last": round(float(np.mean(losses[-100:])), 4),
            "eval": evals,
            "enabled": all(r["learned"]["converged"] and r["learned"]["iterations"] < r["plain"]["iterations"]
                           for r in evals)}


def two_grid_leg():
    """Two-grid spectrum of the coloured multiplicative CAV cycle on the paper's
    N=16 membrane (Section 5.1) for the kappa_s of Table 1, assembled on the
    GPU; the paper's printed values are given beside them as context."""
    from paper_2608_14310_amd import Solver, spectral
    import workloads
    paper = {}
    with open(os.path.join(ROOT, "tests", "golden", "paper_table1.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, r, lo, hi = line.split()
                paper[float(k)] = (float(r), float(lo), float(hi))
    rows = []
    for k in sorted(paper):
        s = workloads.paper_membrane(16, kappa=k)
        s.n_levels = 2
        g = Solver(0)
        g.setup(s, precision="fp64", alpha=1.0, smoother="multiplicative")
        row = {"kappa_s": k}
        for order in ("explicit_first", "standard_first"):
            g.set_phase_order(order)
            sp = spectral.spectrum(spectral.iteration_matrix(g), 16)
            row[order] = {q: round(v, 4) for q, v in sp.items()}
        g.close()
        row["paper"] = dict(zip(("rho_T", "min_abs_lambda", "max_abs_lambda"), paper[k]))
        rows.append(row)
    return rows


def fibre_leg(grids, iterates: int = 3):
    """The clamped flexible fibre of Section 5.3 at the grids of Table 3: for
    each grid a sequence of configurations (straight to strongly bent), each
    a full rebuild of the hierarchy in one context (operator with the fibre's
    tangent law, patches, factors) and a multiplicative-CAV FGMRES solve to
    1e-10, as every Newton linear system needs. The paper's Table 3 row is
    given beside each as context (its counts are averages over a whole
    time-dependent run, not over these configurations). Each grid also times
    one Newton step of the fibre in the downward stream (Section 2 scheme)."""
    import numpy as np
    import torch

    from paper_2608_14310_amd import Solver
    import workloads
    paper = {}
    with open(os.path.join(ROOT, "tests", "golden", "paper_table3.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                v = line.split()
                paper[int(v[0])] = dict(zip(("M", "newton_avg", "fgmres_avg", "fgmres_max", "patch_avg",
                                             "patch_max"), [float(t) for t in v[1:]]))
    rows = []
    for N in grids:
        n_levels = int(round(np.log2(N / 8))) + 1
        g = Solver(0)
        its, t_setup, t_solve = [], [], []
        for q in range(iterates + 1):
            amp = 0.3 * max(q - 1, 0) / max(iterates - 1, 1)
            s = workloads.flexible_fibre(N, n_levels, amp=amp, seed=q)
            bt = torch.from_numpy(s.b).cuda()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.build_operator(s)
            stats = g.build_cav_patches("cav")
            g.factor_patches("fp64", 1e6)
            g.set_smoother("multiplicative", 1.0)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, inf = g.fgmres_solve(bt, rtol=1e-10, max_it=150)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            if q == 0:
                continue  # warm-up: first use of this hierarchy shape
            its.append(inf["iterations"])
            t_setup.append(t1 - t0)
            t_solve.append(t2 - t1)
            assert inf["converged"] == 1, (N, amp)
        # one backward-Euler step of the fibre in the downward stream by
        # Newton's method (hierarchy rebuilt per Newton system, FGMRES 1e-9)
        sn = workloads.flexible_fibre(N, n_levels, amp=0.3, seed=1)
        un = workloads.fibre_inflow_velocity(N, seed=1)
        rhs = torch.from_numpy(np.concatenate([sn.rho / sn.dt * un, np.zeros(N * N)])).cuda()
        g.newton_solve(sn, rhs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, ninf = g.newton_solve(sn, rhs)
        torch.cuda.synchronize()
        t_newton = time.perf_counter() - t0
        g.close()
        fin = stats[-1]
        rows.append({"grid": N, "levels": n_levels, "M": len(s.markers()),
                     "fgmres_its": its, "setup_ms": round(1e3 * float(np.mean(t_setup)), 2),
                     "solve_ms": round(1e3 * float(np.mean(t_solve)), 2),
                     "patch_avg": round(fin["avg_np"], 2), "patch_max": fin["max_np"],
                     "newton_step": {"corrections": ninf["newton_its"], "converged": ninf["converged"],
                                     "fgmres_its_total": ninf["fgmres_its_total"],
                                     "fgmres_its_max": ninf["fgmres_its_max"],
                                     "ms": round(1e3 * t_newton, 2)},
                     "paper": paper.get(N)})
    return rows


def fibre_robustness_leg(N: int = 128):
    """Table 4's parameter rows on the 128² grid: for each (Re, gamma_b,
    gamma_s, gamma_c) one Newton step of the fibre in the downward stream from
    rest (hierarchy rebuilt per Newton system, FGMRES 1e-9) and the largest
    finest-level patch, with the paper's row beside it as context (its counts
    are averages over a whole run)."""
    import numpy as np
    import torch

    from paper_2608_14310_amd import Solver
    import workloads
    rows = []
    with open(os.path.join(ROOT, "tests", "golden", "paper_table4.txt")) as f:
        table = [line.split() for line in f if line.strip() and not line.startswith("#")]
    n_levels = int(round(np.log2(N / 8))) + 1
    g = Solver(0)
    for v in table:
        Re, gb, gs, gc = (float(t) for t in v[:4])
        s = workloads.flexible_fibre(N, n_levels, amp=0.3, seed=1, Re=Re, gamma=(gb, gs, gc))
        un = workloads.fibre_inflow_velocity(N, seed=1)
        rhs = torch.from_numpy(np.concatenate([s.rho / s.dt * un, np.zeros(N * N)])).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, inf = g.newton_solve(s, rhs)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        stats = g.build_cav_patches("cav")
        rows.append({"Re": Re, "gamma": [gb, gs, gc], "corrections": inf["newton_its"],
                     "converged": inf["converged"], "fgmres_its_total": inf["fgmres_its_total"],
                     "fgmres_its_max": inf["fgmres_its_max"], "patch_max": stats[-1]["max_np"],
                     "ms": round(1e3 * (t1 - t0), 2),
                     "paper": dict(zip(("newton_avg", "fgmres_avg", "fgmres_max", "patch_max"),
                                       (float(t) for t in v[4:])))})
    g.close()
    return rows


def box_comparison_leg():
    """CAV against B(b,o) box relaxation on the paper's membrane (Section 5.1):
    two-grid spectral radii of Fig. 2 (N = 32, coarse 16^2) assembled on the
    GPU, and FGMRES iteration counts with V-cycles down to 8^2 at N = 16, 32,
    64 (seeded random right-hand sides; the paper uses the physical first-step
    right-hand side). The paper's values are given beside ours as context."""
    import numpy as np
    import torch

    import workloads
    from paper_2608_14310_amd import Solver, spectral
    fig2, counts = [], {}
    with open(os.path.join(ROOT, "tests", "golden", "paper_box_comparison.txt")) as f:
        for line in f:
            t = line.split()
            if not t or t[0].startswith("#"):
                continue
            if t[0] == "fig2":
                fig2.append((t[1], int(t[2]), int(t[3]), float(t[4]), float(t[5])))
            else:
                counts[int(t[1])] = (int(t[2]), int(t[3]))
    out = {"fig2": [], "fgmres": []}
    for fam, b, o, mu, paper in fig2:
        s = workloads.paper_membrane(32, kappa=1e4, mu=mu)
        s.n_levels = 2
        g = Solver(0)
        family = "cav" if fam == "CAV" else ("vanka" if (b, o) == (1, 0) else "box")
        g.setup(s, family=family, precision="fp64", alpha=1.0, smoother="multiplicative", box=(b, o))
        sp = spectral.spectrum(spectral.iteration_matrix(g), 32)
        g.close()
        out["fig2"].append({"patches": "CAV" if fam == "CAV" else f"B({b},{o})", "mu": mu,
                            "rho_T": round(sp["rho_T"], 3), "paper_rho_T": paper})
    for N, (p_cav, p_box) in sorted(counts.items()):
        s = workloads.paper_membrane(N, kappa=1e4, mu=1e-2)
        s.n_levels = workloads.levels_to(N, 8)
        row = {"N": N, "paper_cav": p_cav, "paper_box42": p_box}
        for fam in ("cav", "box"):
            g = Solver(0)
            g.setup(s, family=fam, precision="fp64", alpha=1.0, smoother="multiplicative", box=(4, 2))
            _, inf = g.fgmres_solve(torch.from_numpy(s.b).to(torch.device("cuda", 0)), 1e-10, 150)
            g.close()
            row["cav" if fam == "cav" else "box42"] = inf["iterations"]
        out["fgmres"].append(row)
    return out


def summarize_counters(path: str):
    """Per kernel and counter of a rocprofv3 counter-collection CSV: the number
    of dispatches and the mean value per dispatch (no GPU needed)."""
    import csv
    tot, cnt = {}, {}
    with open(path) as f:
        for r in csv.DictReader(f):
            k = r["Kernel_Name"].replace("cav::(anonymous namespace)::", "").split("(")[0].replace("void ", "")
            key = (k, r["Counter_Name"])
            tot[key] = tot.get(key, 0.0) + float(r["Counter_Value"])
            cnt[key] = cnt.get(key, 0) + 1
    out = {}
    for (k, c), v in sorted(tot.items()):
        out.setdefault(k, {})[c] = {"dispatches": cnt[(k, c)], "mean": v / cnt[(k, c)]}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--smoother", default="additive", choices=["multiplicative", "additive"],
                    help="smoother of the timed steps: the weighted additive CAV cycle (Appendix A; default "
                         "alpha 0.9, V(3,3)) or the paper's coloured multiplicative V(1,1); the other is timed "
                         "beside it")
    ap.add_argument("--alpha", type=float, default=None, help="damping (default 0.9 additive, 1 multiplicative)")
    ap.add_argument("--sweeps", type=int, default=None,
                    help="pre- and post-sweeps per level (default 3 additive, 1 multiplicative)")
    ap.add_argument("--layout", default="symmetric", choices=["symmetric", "full"],
                    help="storage of the patch inverses for the additive smoother (the multiplicative one always "
                         "reads the full layout)")
    ap.add_argument("--kappa-b", type=float, default=1e-2)
    ap.add_argument("--stiff-sweep", type=float, nargs="*", default=[1.0, 1e2])
    ap.add_argument("--tune", default="default",
                    choices=["default", "auto", "exp1024", "split", "sweep", "coop64", "coop128", "coopr", "coopr1", "coopr0"],
                    help="phase-kernel table of the timed steps: the library's default (the cooperative form "
                         "with a shared residual for every phase), autotuned, one workgroup per patch everywhere "
                         "(exp1024), the split form, the one-launch sweep, or a cooperative form for phases with "
                         "patches over 128 rows (coopr1: over 64 rows, coopr0: all); the autotuned table is "
                         "reported after them")
    ap.add_argument("--no-other-precision", action="store_true")
    ap.add_argument("--no-autotune-report", action="store_true",
                    help="skip the autotuner run reported beside the timed table")
    ap.add_argument("--no-two-grid", action="store_true", help="skip the Table 1 two-grid spectra")
    ap.add_argument("--batch", type=int, default=64, help="systems in the batched leg (0: skip)")
    ap.add_argument("--learned-pairs", type=int, default=600, help="training pairs of the learned leg (0: skip)")
    ap.add_argument("--learned-steps", type=int, default=600)
    ap.add_argument("--learned-c5-eval-precision", default="mixed", choices=["fp64", "mixed"])
    ap.add_argument("--learned-c5", action="store_true",
                    help="the learned stage at its configured scale (20k pairs at 256^2, evaluated at 1024^2); "
                         "not part of the default run")
    ap.add_argument("--multi-rhs", type=int, default=64,
                    help="right-hand sides of the multi-RHS V-cycle leg, blocks of 16 (0: skip)")
    ap.add_argument("--fibre-grids", type=int, nargs="*", default=[],
                    help="grids of the flexible-fibre context leg (Table 3, e.g. 32 64 128 256; default: skip)")
    ap.add_argument("--no-additive", action="store_true", help="skip the weighted additive smoother leg")
    ap.add_argument("--no-paper-v11", action="store_true",
                    help="skip the other smoother's leg (the paper's multiplicative V(1,1) when the timed steps "
                         "are additive)")
    ap.add_argument("--no-membrane", action="store_true",
                    help="skip the 256^2 membrane stiffness leg (FP64 against FP32 factors)")
    ap.add_argument("--additive-only", action="store_true",
                    help="run only the additive V-cycles on the 512^2 beam (for profiling k_add_smooth), then exit")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, help="run only a plain copy of this many bytes")
    ap.add_argument("--calibrate-read", type=int, default=0,
                    help="run only a plain streaming read of this many bytes and print its rate")
    ap.add_argument("--summarize-counters", default="",
                    help="print per-kernel dispatch counts and mean values of a rocprofv3 counter CSV, then exit")
    a = ap.parse_args()
    if a.summarize_counters:
        print(json.dumps(summarize_counters(a.summarize_counters), indent=1))
        return
    if a.calibrate_copy:
        copy_calibration(a.calibrate_copy)
        return
    if a.calibrate_read:
        read_calibration(a.calibrate_read)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus above 1 is not supported"}))
        sys.exit(2)
    if a.additive_only:
        import torch
        print(json.dumps(additive_leg(torch.device("cuda", 0), membrane=False)))
        return

    import numpy as np
    import torch

    import workloads
    from paper_2608_14310_amd import Solver

    global ADD_LAYOUT
    ADD_LAYOUT = a.layout
    layout = _layout(a.smoother)
    dev = torch.device("cuda", 0)
    s = workloads.beam_512(a.kappa_b)
    b = torch.from_numpy(s.b).to(dev)
    g = Solver(0)
    g.set_factor_layout(layout)
    alpha = a.alpha if a.alpha is not None else (1.0 if a.smoother == "multiplicative" else 0.9)
    sweeps = a.sweeps if a.sweeps is not None else (1 if a.smoother == "multiplicative" else 3)
    table = None

    def setup(precision):
        t0 = time.perf_counter()
        g.build_operator(s)
        t1 = time.perf_counter()
        stats = g.build_cav_patches("cav")
        t2 = time.perf_counter()
        fst = g.factor_patches(precision, 1e6)
        g.set_smoother(a.smoother, alpha, sweeps, sweeps)
        if table is not None:
            g.set_tuning(table)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        return dict(build=t1 - t0, patches=t2 - t1, factor=t3 - t2), stats, fst

    def one_step(precision):
        tm, stats, fst = setup(precision)
        g.kernel_timing(True)
        t3 = time.perf_counter()
        x, info = g.fgmres_solve(b, rtol=1e-10, max_it=150)
        torch.cuda.synchronize()
        tm["solve"] = time.perf_counter() - t3
        kt = g.kernel_timing(False)
        return dict(tm, its=info["iterations"], conv=info["converged"], est=info["est_rel_residual"],
                    true=info["true_rel_residual"], stats=stats, fst=fst, kt=kt, x=x)

    # phase-kernel table for this hierarchy shape (outside the timed region)
    setup(a.precision)
    if a.tune == "auto":
        table = g.autotune(reps=3)
    elif a.tune == "split":
        table = np.zeros((s.n_levels, 5), dtype=np.int32)
    elif a.tune == "sweep":
        table = np.full((s.n_levels, 5), 1024, dtype=np.int32)
        table[:, 4] = 1
    elif a.tune == "exp1024":
        table = np.full((s.n_levels, 5), 1024, dtype=np.int32)
        table[:, 4] = 0
    elif a.tune in ("coop64", "coop128", "coopr", "coopr1", "coopr0"):
        table = np.full((s.n_levels, 5), 1024, dtype=np.int32)
        table[:, 4] = 0
        table[:, 2:4] = {"coop64": 1, "coop128": 2, "coopr": 3, "coopr1": 3, "coopr0": 3}[a.tune]
        if a.tune in ("coopr1", "coopr0"):
            table[:, 1] = 3
        if a.tune == "coopr0":
            table[:, 0] = 3
    for _ in range(a.warmup):
        one_step(a.precision)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [one_step(a.precision) for _ in range(a.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1e3 * wall / a.steps

    kernel, kb_bytes, kb_ms, kb_launch = dominant_kernel([r["kt"] for r in runs], a.smoother, a.tune)
    achieved = kb_bytes / (kb_ms * 1e-3) / 1e9 if kb_ms > 0 else 0.0
    last = runs[-1]
    bv = vcycle_bytes(last["stats"], last["fst"], s.N, s.n_levels, a.precision, sweeps)
    solve_ms = [1e3 * r["solve"] for r in runs]
    line = {
        "metric": "FGMRES(CAV-MG) time-to-1e-10 rel. residual at 512^2; V-cycle HBM GB/s",
        "value": round(ms_per_step, 3),
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
        "config": {"workload": f"beam512: 512x512 MAC grid, 5-level V({sweeps},{sweeps}) CAV multigrid "
                               f"({a.smoother} smoother, alpha {alpha:g}), 4 open fibres L=0.4 "
                               f"ds=h/2, kappa_b={a.kappa_b:g}, kappa_s=1e4, rho=1 mu=0.01 dt=1e-3, seeded U[-1,1] "
                               "RHS, FGMRES rtol 1e-10; value = T_total (operator + patches + factors + solve)",
                   "precision": a.precision, "smoother": a.smoother, "alpha": alpha, "sweeps": sweeps,
                   "factor_layout": layout, "tune": a.tune},
        "t_solve_ms": round(float(np.median(solve_ms)), 3),
        "per_step": {k: (float("%.4g" % v) if isinstance(v, float) else v) for k, v in last.items()
                     if k not in ("stats", "fst", "kt", "x")},
        "vcycle_ms": round(last["kt"]["vcycle_ms"], 4),
        "vcycles_per_s": round(1e3 / last["kt"]["vcycle_ms"], 1) if last["kt"]["vcycle_ms"] else None,
        "vcycle_bytes": int(bv),
        "vcycle_gbs": round(bv / (last["kt"]["vcycle_ms"] * 1e-3) / 1e9, 1) if last["kt"]["vcycle_ms"] else None,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(kernel, a.precision, a.smoother, a.tune, layout),
                     "kernel": kernel, "launches": kb_launch,
                     "bytes_per_launch": int(kb_bytes / max(kb_launch, 1)),
                     "avg_launch_us": round(1e3 * kb_ms / max(kb_launch, 1), 3)},
    }
    line["solves_per_s"] = round(1e3 / ms_per_step, 2)
    # the read rate a plain stream reaches on this part, over the size of the
    # stored inverses (far beyond the last-level cache)
    rc = measure_read(int(max(last["fst"]["factor_bytes"], 1 << 28)))
    line["read_calibration"] = dict(rc, what="torch.sum over float64 of the stored factor bytes of all levels")
    if last["kt"]["vcycle_ms"]:
        line["vcycle_frac_of_read"] = round(bv / (last["kt"]["vcycle_ms"] * 1e-3) / 1e9 / rc["read_gbs"], 4)
    line["roofline"]["frac_of_read"] = round(achieved / rc["read_gbs"], 4)
    if table is not None:
        line["tuning_table"] = np.asarray(table).tolist()
    if a.smoother == "multiplicative" and a.tune != "auto" and not a.no_autotune_report:
        # the autotuner on the same hierarchy, reported beside the timed table
        setup(a.precision)
        tuned = g.autotune(reps=3)
        torch.cuda.synchronize()
        t0a = time.perf_counter()
        _, inf = g.fgmres_solve(b, rtol=1e-10, max_it=150)
        torch.cuda.synchronize()
        line["autotune"] = {"table": np.asarray(tuned).tolist(), "its": inf["iterations"],
                            "t_solve_ms": round(1e3 * (time.perf_counter() - t0a), 1)}
    # the other precision, same workload, for comparison
    other = "mixed" if a.precision == "fp64" else "fp64"
    if not a.no_other_precision:
        o = one_step(other)
        x64, xo = (last["x"], o["x"]) if a.precision == "fp64" else (o["x"], last["x"])
        line["other_precision"] = {
            "precision": other, "t_total_ms": round(1e3 * (o["build"] + o["patches"] + o["factor"] + o["solve"]), 1),
            "t_solve_ms": round(1e3 * o["solve"], 1), "its": o["its"], "true": o["true"],
            "rel_err_vs_fp64": float("%.3g" % (torch.linalg.norm(xo - x64) / torch.linalg.norm(x64)).item()),
            "n_fp32_patches": o["fst"]["n_fp32"], "n_fp64_patches": o["fst"]["n_fp64"]}
        del o
    if not a.no_membrane:
        line["membrane256"] = membrane_leg(dev)
    if not a.no_paper_v11:
        other_sm = "multiplicative" if a.smoother == "additive" else "additive"
        line["multiplicative_v11" if other_sm == "multiplicative" else "additive_v33"] = (
            paper_v11_leg(dev, a.kappa_b) if other_sm == "multiplicative" else additive_sweeps_leg(dev))
    if a.multi_rhs > 0:
        # the V-cycle on blocks of 16 right-hand sides (explicit phases as FP64
        # MFMA products) against one cycle per column, outside the timed steps
        g.set_factor_layout("full")
        setup(a.precision)
        g.set_smoother("multiplicative", 1.0)
        gen = torch.Generator(device=dev)
        gen.manual_seed(5)
        R = torch.randn((a.multi_rhs, b.numel()), generator=gen, dtype=torch.float64, device=dev)
        g.vcycle_multi(R[:16])
        g.vcycle(R[0])
        torch.cuda.synchronize()
        t0m = time.perf_counter()
        Z = g.vcycle_multi(R)
        torch.cuda.synchronize()
        tm = time.perf_counter() - t0m
        t0c = time.perf_counter()
        Zs = [g.vcycle(R[q]) for q in range(a.multi_rhs)]
        torch.cuda.synchronize()
        tc = time.perf_counter() - t0c
        diff = max(float((Z[q] - Zs[q]).abs().max() / Zs[q].abs().max()) for q in range(a.multi_rhs))
        line["multi_rhs"] = {"columns": a.multi_rhs, "block": 16,
                             "ms_per_column": round(1e3 * tm / a.multi_rhs, 3),
                             "single_cycle_ms_per_column": round(1e3 * tc / a.multi_rhs, 3),
                             "speedup": round(tc / tm, 2), "max_rel_diff_vs_single": float("%.3g" % diff)}
        g.set_factor_layout(layout)
    if a.fibre_grids:
        line["fibre"] = fibre_leg(a.fibre_grids)
        line["fibre_robustness"] = fibre_robustness_leg()
    gpu_full = {}
    if not a.no_additive:
        line["additive"] = additive_leg(dev)
        gpu_full["membrane256"] = line["additive"]["membrane256"]["additive"]
    # the 32^2 target system (additive cycle), for the CPU comparison
    if not a.no_cpu_baseline:
        st32 = workloads.small_target(0)
        g32 = Solver(0)
        g32.setup(st32, precision="fp64", alpha=0.7, smoother="additive", layout=_layout("additive"))
        b32 = torch.from_numpy(st32.b).to(dev)
        g32.fgmres_solve(b32, rtol=1e-10, max_it=150)
        torch.cuda.synchronize()
        t0c = time.perf_counter()
        g32.build_operator(st32)
        g32.build_cav_patches("cav")
        g32.factor_patches("fp64", 1e6)
        g32.set_smoother("additive", 0.7)
        t1c = time.perf_counter()
        _, inf32 = g32.fgmres_solve(b32, rtol=1e-10, max_it=150)
        torch.cuda.synchronize()
        t2c = time.perf_counter()
        g32.close()
        gpu_full["target32"] = {"iterations": inf32["iterations"], "t_total_ms": round(1e3 * (t2c - t0c), 2),
                                "t_solve_ms": round(1e3 * (t2c - t1c), 2)}
    sweep = []
    for kb in a.stiff_sweep:
        sk = workloads.beam_512(kb)
        g.build_operator(sk)
        g.build_cav_patches("cav")
        row = {"kappa_b": kb}
        for sm, al, sw in ((a.smoother, alpha, sweeps), ("multiplicative", 1.0, 1)):
            key = f"{sm}_v{sw}{sw}"
            if key in row:
                continue
            g.set_factor_layout(_layout(sm))
            g.factor_patches(a.precision, 1e6)
            g.set_smoother(sm, al, sw, sw)
            t0s = time.perf_counter()
            _, inf = g.fgmres_solve(torch.from_numpy(sk.b).to(dev), rtol=1e-10, max_it=150)
            torch.cuda.synchronize()
            row[key] = {"iterations": inf["iterations"], "converged": inf["converged"],
                        "est_rel_residual": float("%.4g" % inf["est_rel_residual"]),
                        "solve_ms": round(1e3 * (time.perf_counter() - t0s), 1)}
        sweep.append(row)
    line["stiffness_sweep"] = sweep
    if a.learned_pairs > 0:
        g.set_factor_layout("full")
        setup("mixed")
        g.set_smoother("multiplicative", 1.0)
        line["learned"] = learned_leg(g, b, a.learned_pairs, a.learned_steps)
    if a.learned_c5:
        line["learned_c5"] = learned_c5_leg(dev, eval_precision=a.learned_c5_eval_precision)
    if not a.no_two_grid:
        line["two_grid_table1"] = two_grid_leg()
        line["box_comparison"] = box_comparison_leg()
    if a.verbose:
        line["level_stats"] = last["stats"]
        line["factor_stats"] = last["fst"]
    g.close()
    if a.batch > 0:
        line["batched"] = batched_leg(a.batch, 150)
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(a.kappa_b, last["its"], a.smoother, gpu_full, alpha=alpha,
                                            sweeps=sweeps)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
