"""Benchmark: CAV-multigrid FGMRES time-to-1e-10 at 512^2 (beam law, 5 levels).

One step = the whole path on the 512^2 open-fibre beam system (4 fibres of
length 0.4, ds = h/2, bending kappa_b = 1e-2, springs 1e4, 5-level V(1,1)):
build_operator -> build_cav_patches -> factor_patches -> fgmres_solve to 1e-10.
`value` is the mean wall time per step (T_total, ms, lower is better);
`t_solve_ms` is the solve alone. Inputs (markers, RHS on the device) are
prepared before the timed region; the phase kernels follow the library's
default table (the cooperative form with a shared residual; the autotuned
table is measured and reported after the timed steps). The dominant kernel
(explicit-patch phase kernel of the multiplicative smoother) is timed live
with HIP events on the library stream around each run of phase launches.
After the timed steps: the other precision on the same system, the stiffer
kappa_b values (reported with their iteration counts), the learned stage
(trained on 256^2 pairs, judged on this solve), the batched mix of independent
systems in one captured graph, and the CPU oracle on a bounded sample.
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


def measured_traffic(kernel: str, precision: str, smoother: str, tune: str):
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
    if not rec or rec["precision"] != precision or rec["smoother"] != smoother or rec.get("tune", "default") != tune:
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
    ap.add_argument("--smoother", default="multiplicative", choices=["multiplicative", "additive"])
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
    ap.add_argument("--multi-rhs", type=int, default=64,
                    help="right-hand sides of the multi-RHS V-cycle leg, blocks of 16 (0: skip)")
    ap.add_argument("--fibre-grids", type=int, nargs="*", default=[32, 64, 128, 256],
                    help="grids of the flexible-fibre leg (Table 3); none: skip")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, help="run only a plain copy of this many bytes")
    ap.add_argument("--summarize-counters", default="",
                    help="print per-kernel dispatch counts and mean values of a rocprofv3 counter CSV, then exit")
    a = ap.parse_args()
    if a.summarize_counters:
        print(json.dumps(summarize_counters(a.summarize_counters), indent=1))
        return
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
    s = workloads.beam_512(a.kappa_b)
    b = torch.from_numpy(s.b).to(dev)
    g = Solver(0)
    alpha = 1.0 if a.smoother == "multiplicative" else 0.7
    table = None

    def setup(precision):
        t0 = time.perf_counter()
        g.build_operator(s)
        t1 = time.perf_counter()
        stats = g.build_cav_patches("cav")
        t2 = time.perf_counter()
        fst = g.factor_patches(precision, 1e6)
        g.set_smoother(a.smoother, alpha)
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
                    true=info["true_rel_residual"], stats=stats, fst=fst, kt=kt)

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

    # the dominant explicit-patch kernel: the shared-residual form when its
    # brackets hold most of the time, else the other cooperative forms, else
    # the one-workgroup form
    co_ms = sum(r["kt"]["coop_ms"] for r in runs)
    sh_ms = sum(r["kt"]["shared_ms"] for r in runs)
    all_ms = sum(r["kt"]["ms"] for r in runs)
    if sh_ms > all_ms - sh_ms:
        kernel = "k_mult_coopr"
        kb_bytes = sum(r["kt"]["shared_bytes"] for r in runs)
        kb_ms = sh_ms
        kb_launch = sum(r["kt"]["shared_launches"] for r in runs)
    elif co_ms > all_ms - co_ms:
        kernel = {"coop64": "k_mult_coop<64>", "coop128": "k_mult_coop<128>"}.get(a.tune, "k_mult_coop")
        kb_bytes = sum(r["kt"]["coop_bytes"] - r["kt"]["shared_bytes"] for r in runs)
        kb_ms = co_ms - sh_ms
        kb_launch = sum(r["kt"]["coop_launches"] - r["kt"]["shared_launches"] for r in runs)
    else:
        kernel = "k_mult_exp" if a.smoother == "multiplicative" else "k_patch_apply"
        kb_bytes = sum(r["kt"]["bytes"] - r["kt"]["coop_bytes"] for r in runs)
        kb_ms = all_ms - co_ms
        kb_launch = sum(r["kt"]["launches"] - r["kt"]["coop_launches"] for r in runs)
    achieved = kb_bytes / (kb_ms * 1e-3) / 1e9 if kb_ms > 0 else 0.0
    last = runs[-1]
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
        "config": {"workload": "beam512: 512x512 MAC grid, 5-level V(1,1) CAV multigrid, 4 open fibres L=0.4 "
                               f"ds=h/2, kappa_b={a.kappa_b:g}, kappa_s=1e4, rho=1 mu=0.01 dt=1e-3, seeded U[-1,1] "
                               "RHS, FGMRES rtol 1e-10; value = T_total (operator + patches + factors + solve)",
                   "precision": a.precision, "smoother": a.smoother, "alpha": alpha, "tune": a.tune},
        "t_solve_ms": round(float(np.median(solve_ms)), 3),
        "per_step": {k: (float("%.4g" % v) if isinstance(v, float) else v) for k, v in last.items()
                     if k not in ("stats", "fst", "kt")},
        "vcycle_ms": round(last["kt"]["vcycle_ms"], 4),
        "vcycles_per_s": round(1e3 / last["kt"]["vcycle_ms"], 1) if last["kt"]["vcycle_ms"] else None,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(kernel, a.precision, a.smoother, a.tune),
                     "kernel": kernel, "launches": kb_launch,
                     "bytes_per_launch": int(kb_bytes / max(kb_launch, 1)),
                     "avg_launch_us": round(1e3 * kb_ms / max(kb_launch, 1), 3)},
    }
    if table is not None:
        line["tuning_table"] = np.asarray(table).tolist()
    if a.tune != "auto" and not a.no_autotune_report:
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
        line["other_precision"] = {
            "precision": other, "t_total_ms": round(1e3 * (o["build"] + o["patches"] + o["factor"] + o["solve"]), 1),
            "t_solve_ms": round(1e3 * o["solve"], 1), "its": o["its"], "true": o["true"],
            "n_fp32_patches": o["fst"]["n_fp32"], "n_fp64_patches": o["fst"]["n_fp64"]}
    if a.multi_rhs > 0:
        # the V-cycle on blocks of 16 right-hand sides (explicit phases as FP64
        # MFMA products) against one cycle per column, outside the timed steps
        setup(a.precision)
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
    if a.fibre_grids:
        line["fibre"] = fibre_leg(a.fibre_grids)
        line["fibre_robustness"] = fibre_robustness_leg()
    sweep = []
    for kb in a.stiff_sweep:
        sk = workloads.beam_512(kb)
        g.build_operator(sk)
        g.build_cav_patches("cav")
        g.factor_patches(a.precision, 1e6)
        g.set_smoother(a.smoother, alpha)
        t0s = time.perf_counter()
        _, inf = g.fgmres_solve(torch.from_numpy(sk.b).to(dev), rtol=1e-10, max_it=150)
        torch.cuda.synchronize()
        sweep.append({"kappa_b": kb, "iterations": inf["iterations"], "converged": inf["converged"],
                      "est_rel_residual": float("%.4g" % inf["est_rel_residual"]),
                      "solve_ms": round(1e3 * (time.perf_counter() - t0s), 1)})
    line["stiffness_sweep"] = sweep
    if a.learned_pairs > 0:
        setup("mixed")
        line["learned"] = learned_leg(g, b, a.learned_pairs, a.learned_steps)
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
        line["cpu_baseline"] = cpu_baseline(a.kappa_b, last["its"], a.smoother, alpha)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
