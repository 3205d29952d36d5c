"""Writes oracle-only expected values for the GPU parity tests at full size.

Runs the FP64 CPU oracle (`oracle/`) on a seeded workload (`workloads/`) and
stores the FGMRES iteration count, the residual history and checksums of the
solution: its 2-norm, its infinity norm, and the entries at 64 seeded
positions (drawn from default_rng(12345) over the vector). Nothing here reads
the GPU path. The CPU time is long (minutes per V-cycle at 512^2), so each
configuration is one invocation:

  python tests/golden/make_goldens.py beam512 KAPPA_B ORDER
      4 open fibres on a 512^2 grid, 5 levels, multiplicative CAV V(1,1)
      (alpha 1) in the coloured ORDER (explicit_first | standard_first),
      FGMRES to 1e-10 (max 150)
  python tests/golden/make_goldens.py membrane256 KAPPA_S SMOOTHER [ORDER]
      ellipse membrane on a 256^2 grid, coarsest 8^2, SMOOTHER additive
      (alpha 0.7, Theta = 1/cnt) or multiplicative (alpha 1, coloured ORDER,
      default explicit_first), FGMRES to 1e-10 (max 150)
  python tests/golden/make_goldens.py additive SYSTEM STIFFNESS ALPHA SWEEPS
      SYSTEM beam512 (kappa_b = STIFFNESS) or membrane256 (kappa_s =
      STIFFNESS), weighted additive CAV (Theta = 1/cnt) with damping ALPHA
      and V(SWEEPS, SWEEPS), FGMRES to 1e-10 (max 150)

Output: tests/golden/<name>.json
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import krylov, multigrid  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
N_SAMPLES = 64


def sample_positions(n: int) -> np.ndarray:
    return np.sort(np.random.default_rng(12345).choice(n, N_SAMPLES, replace=False))


def run(system, smoother: str, alpha: float, order: str, name: str, meta: dict, sweeps: int = 1) -> dict:
    t0 = time.time()
    if smoother == "multiplicative":
        H = multigrid.Hierarchy(system, alpha=alpha, smoother="coloured", order=order, pre=sweeps, post=sweeps)
    else:
        H = multigrid.Hierarchy(system, alpha=alpha, smoother="additive", pre=sweeps, post=sweeps)
    t_setup = time.time() - t0
    K = H.levels[-1].K
    count = [0]

    def prec(v):
        count[0] += 1
        print(f"{name}: V-cycle {count[0]} at {time.time() - t0:.0f} s", flush=True)
        return H.vcycle(v)

    res = krylov.fgmres(lambda z: K @ z, prec, system.b, 1e-10, 150)
    x = res.x
    pos = sample_positions(x.size)
    out = dict(meta, name=name, N=system.N, n_levels=system.n_levels, smoother=smoother, alpha=alpha,
               order=order if smoother == "multiplicative" else None, pre=sweeps, post=sweeps,
               rtol=1e-10, max_it=150,
               iterations=res.iterations, converged=bool(res.converged), history=[float(h) for h in res.history],
               true_rel_residual=float(np.linalg.norm(system.b - K @ x) / np.linalg.norm(system.b)),
               x_norm2=float(np.linalg.norm(x)), x_norminf=float(np.abs(x).max()),
               sample_positions=pos.tolist(), sample_values=[float(v) for v in x[pos]],
               oracle_setup_s=round(t_setup, 1), oracle_total_s=round(time.time() - t0, 1))
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps({k: out[k] for k in ("name", "iterations", "converged", "true_rel_residual")}), flush=True)
    return out


def main(argv):
    kind = argv[0]
    if kind == "beam512":
        kb, order = float(argv[1]), argv[2]
        s = workloads.beam_512(kb, seed=0)
        run(s, "multiplicative", 1.0, order, f"beam512_kb{kb:g}_{order}",
            dict(workload="beam_512", kappa_b=kb, seed=0))
    elif kind == "membrane256":
        ks, smoother = float(argv[1]), argv[2]
        order = argv[3] if len(argv) > 3 else "explicit_first"
        s = workloads.membrane_256(ks, seed=0)
        alpha = 0.7 if smoother == "additive" else 1.0
        tag = smoother if smoother == "additive" else f"{smoother}_{order}"
        run(s, smoother, alpha, order, f"membrane256_ks{ks:g}_{tag}",
            dict(workload="membrane_256", kappa_s=ks, seed=0))
    elif kind == "additive":
        system, k, alpha, sweeps = argv[1], float(argv[2]), float(argv[3]), int(argv[4])
        if system == "beam512":
            s = workloads.beam_512(k, seed=0)
            meta = dict(workload="beam_512", kappa_b=k, seed=0)
            stem = f"beam512_kb{k:g}"
        elif system == "membrane256":
            s = workloads.membrane_256(k, seed=0)
            meta = dict(workload="membrane_256", kappa_s=k, seed=0)
            stem = f"membrane256_ks{k:g}"
        else:
            raise SystemExit(__doc__)
        run(s, "additive", alpha, "", f"{stem}_additive_a{alpha:g}_v{sweeps}{sweeps}", meta, sweeps)
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
