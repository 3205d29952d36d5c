"""FGMRES on the full-size configurations against expected values written by
the oracle alone (`tests/golden/make_goldens.py`): the 512^2 beam of the
headline measurement and the 256^2 membrane at kappa_s = 1e2, 1e4, 1e6, with
the paper's V(1,1) cycles and with the additive cycle's V(3,3) form.

Iteration counts must be identical (the GPU and the oracle run the same
cycle; the FP64 rounding of the explicit inverses stays far below what moves
the count). The solution must agree with the oracle's to 1e-8 relative, checked
on its 2-norm and on 64 seeded entries (relative to the infinity norm), and the
true relative residual must be at most 2e-10 (or, where the oracle itself
stops at the FP64 rounding floor of a very stiff system, within 3x of the
oracle's and flagged FLOOR_LIMITED). Mixed precision (FP32 factors of
well-conditioned patches, FP64 elsewhere) is run on the same systems; its
iteration count and its error against the FP64 oracle solution are reported
per solve, and it must meet the same residual.
"""
import glob
import json
import os

import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
GOLDENS = sorted(glob.glob(os.path.join(HERE, "beam512_*.json")) + glob.glob(os.path.join(HERE, "membrane256_*.json")))


def _system(g):
    if g["workload"] == "beam_512":
        return workloads.beam_512(g["kappa_b"], seed=g["seed"])
    return workloads.membrane_256(g["kappa_s"], seed=g["seed"])


def _solve(g, precision, layout="full"):
    from paper_2608_14310_amd import Solver
    s = _system(g)
    sol = Solver(0)
    try:
        sol.setup(s, precision=precision, alpha=g["alpha"], smoother=g["smoother"], layout=layout)
        sweeps = g.get("pre", 1)
        sol.set_smoother(g["smoother"], g["alpha"], sweeps, g.get("post", sweeps))
        if g["smoother"] == "multiplicative":
            sol.set_phase_order(g["order"])
        x, info = sol.fgmres_solve(torch.from_numpy(s.b).cuda(), rtol=g["rtol"], max_it=g["max_it"])
        torch.cuda.synchronize()
        return x.cpu().numpy(), info
    finally:
        sol.close()


def _errors(x, g):
    pos = np.asarray(g["sample_positions"])
    ref = np.asarray(g["sample_values"])
    e_norm = abs(np.linalg.norm(x) - g["x_norm2"]) / g["x_norm2"]
    e_samp = np.abs(x[pos] - ref).max() / g["x_norminf"]
    return e_norm, e_samp


ADDITIVE = [p for p in GOLDENS if "_additive" in os.path.basename(p)]


@pytest.mark.parametrize("path", GOLDENS, ids=[os.path.basename(p)[:-5] for p in GOLDENS])
def test_fgmres_matches_oracle_golden(path):
    _check_fp64(path, "full")


@pytest.mark.parametrize("path", ADDITIVE, ids=[os.path.basename(p)[:-5] for p in ADDITIVE])
def test_symmetric_layout_matches_oracle_golden(path):
    """The additive cycles with the patch inverses in the symmetric panel
    layout (lower panels stored, upper entries mirrored): the same bounds."""
    _check_fp64(path, "symmetric")


def _check_fp64(path, layout):
    with open(path) as f:
        g = json.load(f)
    print(f"[golden] {g['name']} ({layout} layout): oracle {g['iterations']} iterations", flush=True)
    x, info = _solve(g, "fp64", layout)
    e_norm, e_samp = _errors(x, g)
    print(f"[golden] {g['name']} fp64 {layout}: {info['iterations']} iterations, true {info['true_rel_residual']:.2e}, "
          f"norm err {e_norm:.1e}, sampled err {e_samp:.1e}", flush=True)
    assert info["converged"] == int(g["converged"])
    assert info["iterations"] == g["iterations"]
    floor = g["converged"] and g["true_rel_residual"] > 2e-10
    np.testing.assert_allclose(info["history"], g["history"], rtol=1e-3 if floor else 1e-5, atol=1e-13)
    if floor:
        # the estimate met 1e-10 but the FP64 rounding floor of this stiff
        # system keeps the oracle's true residual above 2e-10; the GPU's sits
        # at the same floor (flagged FLOOR_LIMITED above 10 rtol)
        assert info["status"] == (101 if info["true_rel_residual"] > 10 * g["rtol"] else 0)
        assert info["true_rel_residual"] <= 3 * g["true_rel_residual"]
        assert e_samp <= 1e-6
    elif g["converged"]:
        assert info["true_rel_residual"] <= 2e-10
        assert e_norm <= 1e-8 and e_samp <= 1e-8
    else:
        # both stop at max_it with the same residual history; a stagnating
        # Krylov space leaves the iterate itself ill-determined
        assert abs(info["true_rel_residual"] - g["true_rel_residual"]) <= 1e-6 * g["true_rel_residual"]


@pytest.mark.parametrize("path", GOLDENS, ids=[os.path.basename(p)[:-5] for p in GOLDENS])
def test_mixed_precision_against_oracle_golden(path):
    with open(path) as f:
        g = json.load(f)
    if not g["converged"]:
        pytest.skip("the FP64 oracle does not converge on this system within max_it")
    floor = g["true_rel_residual"] > 2e-10
    x, info = _solve(g, "mixed")
    e_norm, e_samp = _errors(x, g)
    print(f"[golden] {g['name']} mixed: {info['iterations']} iterations (FP64 oracle {g['iterations']}), "
          f"true {info['true_rel_residual']:.2e}, error against the FP64 oracle: norm {e_norm:.1e}, "
          f"sampled {e_samp:.1e}", flush=True)
    assert info["converged"] == 1
    assert info["true_rel_residual"] <= (3 * g["true_rel_residual"] if floor else 2e-10)
    # two solutions that each meet a 1e-10 relative residual differ by at most
    # about cond(K_E) * 2e-10; these systems stay within 1e-6 of each other
    assert e_samp <= 1e-6
