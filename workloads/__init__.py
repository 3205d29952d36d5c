"""Seeded synthetic problem instances shaped like the paper's model problems.

This package holds problem *data* only: grid size, fluid parameters, Lagrangian
marker positions and quadrature weights, the chosen force law with its
stiffness values, and the right-hand side. It contains none of the method's
arithmetic (no operators, kernels, patches or solvers). Both the CPU oracle and
the GPU path take their inputs from here.

Geometry follows the paper's model problems (Section 5): a periodic unit
square, Lagrangian spacing about h/2 (Section 5.1), markers equally spaced in
arclength, quadrature weight omega_k = ds (Appendix A). Right-hand sides are
i.i.d. uniform[-1, 1] with the pressure block shifted to mean zero, because the
reduced operator's range excludes constant pressure (Section 5.1, gauge mode).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

LAWS = ("target", "membrane", "beam_open", "beam_closed", "fibre")


@dataclasses.dataclass
class Segment:
    """One Lagrangian curve: markers X (M x 2, in [0,1)^2), closed or open,
    uniform spacing ds (the quadrature weight of every marker)."""
    X: np.ndarray
    closed: bool
    ds: float


@dataclasses.dataclass
class System:
    """One reduced Eulerian IB system: grid, fluid parameters, structure, RHS."""
    name: str
    N: int
    n_levels: int
    rho: float
    mu: float
    dt: float
    law: str
    kappa: Dict[str, float]
    segments: List[Segment]
    b: np.ndarray  # length 3 N^2, layout [u | v | p], each block [i][j] (j fastest)

    @property
    def M(self) -> int:
        return sum(len(s.X) for s in self.segments)

    @property
    def n(self) -> int:
        return 3 * self.N * self.N

    def markers(self) -> np.ndarray:
        return np.concatenate([s.X for s in self.segments], axis=0)

    def weights(self) -> np.ndarray:
        return np.concatenate([np.full(len(s.X), s.ds) for s in self.segments])


# ---------------------------------------------------------------- geometry ---

def circle(cx: float, cy: float, r: float, spacing: float) -> Segment:
    M = int(round(2.0 * math.pi * r / spacing))
    th = 2.0 * math.pi * np.arange(M) / M
    X = np.stack([cx + r * np.cos(th), cy + r * np.sin(th)], axis=1)
    return Segment(np.mod(X, 1.0), True, 2.0 * math.pi * r / M)


def _closed_curve_equal_arclength(fx, fy, spacing: float, samples: int = 1 << 18) -> Segment:
    """Markers equally spaced in arclength along a closed parametric curve
    t in [0, 2pi), located by dense sampling and linear interpolation."""
    t = np.linspace(0.0, 2.0 * math.pi, samples + 1)
    x, y = fx(t), fy(t)
    seg = np.hypot(np.diff(x), np.diff(y))
    s = np.concatenate([[0.0], np.cumsum(seg)])
    P = float(s[-1])
    M = int(round(P / spacing))
    ds = P / M
    tk = np.interp(np.arange(M) * ds, s, t)
    X = np.stack([fx(tk), fy(tk)], axis=1)
    return Segment(np.mod(X, 1.0), True, ds)


def ellipse(cx: float, cy: float, ax: float, ay: float, spacing: float) -> Segment:
    return _closed_curve_equal_arclength(lambda t: cx + ax * np.cos(t),
                                         lambda t: cy + ay * np.sin(t), spacing)


def trefoil_radius_curve(cx: float, cy: float, r0: float, r1: float, spacing: float) -> Segment:
    """Closed curve r(theta) = r0 + r1 cos(3 theta) (the paper's beam test shape)."""
    return _closed_curve_equal_arclength(lambda t: cx + (r0 + r1 * np.cos(3 * t)) * np.cos(t),
                                         lambda t: cy + (r0 + r1 * np.cos(3 * t)) * np.sin(t), spacing)


def open_fibre(cx: float, cy: float, angle: float, length: float, spacing: float) -> Segment:
    M = int(round(length / spacing)) + 1
    ds = length / (M - 1)
    s = np.arange(M) * ds - 0.5 * length
    X = np.stack([cx + s * math.cos(angle), cy + s * math.sin(angle)], axis=1)
    return Segment(np.mod(X, 1.0), False, ds)


def row_of_markers(y: float, spacing: float) -> Segment:
    """A horizontal periodic row of markers (the paper's target-point walls)."""
    M = int(round(1.0 / spacing))
    X = np.stack([np.arange(M) / M, np.full(M, y)], axis=1)
    return Segment(X, True, 1.0 / M)


def random_rhs(N: int, seed: int) -> np.ndarray:
    b = np.random.default_rng(seed).uniform(-1.0, 1.0, 3 * N * N)
    p = b[2 * N * N:]
    p -= p.mean()
    return b


# ----------------------------------------------------------------- systems ---

FLUID = dict(rho=1.0, mu=0.01, dt=1e-3)


def levels_to(N: int, coarsest: int) -> int:
    L = 1
    while (N >> (L - 1)) > coarsest:
        L += 1
    assert N >> (L - 1) == coarsest, (N, coarsest)
    return L


def target_circle(N: int = 32, n_levels: int = 3, kappa: float = 1e4, seed: int = 0,
                  **fluid) -> System:
    """Target-point law on a circle of radius 0.25 centred in the unit square."""
    h = 1.0 / N
    f = dict(FLUID, **fluid)
    seg = circle(0.5, 0.5, 0.25, h / 2)
    return System(f"target_circle_N{N}_k{kappa:g}_s{seed}", N, n_levels, f["rho"], f["mu"], f["dt"],
                  "target", {"kappa_t": kappa}, [seg], random_rhs(N, seed))


def membrane_ellipse(N: int = 256, n_levels: Optional[int] = None, kappa: float = 1e4, seed: int = 0,
                     ax: float = 0.2, ay: float = 0.15, **fluid) -> System:
    """Closed elastic membrane (nearest-neighbour springs) on an ellipse."""
    h = 1.0 / N
    f = dict(FLUID, **fluid)
    L = n_levels if n_levels is not None else levels_to(N, 8)
    seg = ellipse(0.5, 0.5, ax, ay, h / 2)
    return System(f"membrane_ellipse_N{N}_k{kappa:g}_s{seed}", N, L, f["rho"], f["mu"], f["dt"],
                  "membrane", {"kappa_s": kappa}, [seg], random_rhs(N, seed))


def beam_fibres(N: int = 512, n_levels: int = 5, kappa_b: float = 1.0, kappa_s: float = 1e4,
                n_fibres: int = 4, length: float = 0.4, seed: int = 0, **fluid) -> System:
    """Open fibres with bending (second differences) plus stretching springs.
    Centres ~ U[0,1)^2 and angles ~ U[0,pi) from the geometry stream
    default_rng([seed, 1]); fibres wrap periodically and may overlap."""
    h = 1.0 / N
    f = dict(FLUID, **fluid)
    g = np.random.default_rng([seed, 1])
    segs = []
    for _ in range(n_fibres):
        cx, cy = g.uniform(0.0, 1.0, 2)
        ang = g.uniform(0.0, math.pi)
        segs.append(open_fibre(cx, cy, ang, length, h / 2))
    return System(f"beam_fibres_N{N}_kb{kappa_b:g}_s{seed}", N, n_levels, f["rho"], f["mu"], f["dt"],
                  "beam_open", {"kappa_b": kappa_b, "kappa_s": kappa_s}, segs, random_rhs(N, seed))


def flexible_fibre(N: int = 64, n_levels: int = 4, amp: float = 0.3, seed: int = 0, Re: float = 200.0,
                   gamma=(1.0, 1.0, 1.0), **fluid) -> System:
    """The clamped flexible fibre of Section 5.3 mapped into the periodic unit
    square by similarity: the paper's (0,2)^2 cell, lengths and times scaled
    by 1/2 with the velocity scale, Reynolds number and energy scale kept.
    Fibre length 0.1875 (paper 0.375), midpoint clamp at (0.5, 0.75) (paper
    (1, 1.5)), markers ds = h/2 apart, so the fibre has the paper's marker
    count at the same N. Bent configuration such as a Newton iterate would
    give: midline y = 0.75 - amp s^2 / L (s the signed arclength from the
    midpoint) plus seeded jitter of 5% of ds per coordinate from
    default_rng([seed, 2]); coordinates unwrapped (the fibre lies inside the
    cell). Stiffness: the paper's EI = 2.63672e-2 and, on its 128 x 128
    grid (h = 1/64 in its cell), K_s, K_p, K_t = 375, 1200, 7.03125, each
    doubled per halving of h (so times N/128 here), then mapped by the
    length scale s = 1/2 through the energy dimensions: EI s^3, K_s s, K_p,
    K_t s^2. Fluid: rho = 1,
    mu = 1.875e-3 s (paper Re kept), dt = 0.05 h (the paper's dt/h). The
    law's parameters ride in `kappa` (EI, K_s, K_p, K_t, clamp marker m,
    clamp point). Table 4's variations: Re (mu scaled by 200 / Re) and
    gamma = (gamma_b, gamma_s, gamma_c) multiplying EI, K_s and both clamp
    penalties."""
    h = 1.0 / N
    ds = h / 2
    sc = 0.5
    L = 0.375 * sc
    M = int(round(L / ds)) + 1
    m = M // 2
    s = (np.arange(M) - m) * ds
    X = np.stack([0.5 + s, 0.75 - amp * s ** 2 / L], axis=1)
    X = X + np.random.default_rng([seed, 2]).uniform(-0.05, 0.05, X.shape) * ds
    refine = N / 128.0
    gb, gs, gc = gamma
    kappa = {"EI": 2.63672e-2 * sc ** 3 * gb, "K_s": 375.0 * refine * sc * gs, "K_p": 1200.0 * refine * gc,
             "K_t": 7.03125 * refine * sc ** 2 * gc, "m": m, "clamp_x": 0.5, "clamp_y": 0.75}
    f = dict(FLUID, mu=1.875e-3 * sc * 200.0 / Re, dt=0.05 * h)
    f.update(fluid)
    return System(f"flexible_fibre_N{N}_a{amp:g}_s{seed}", N, n_levels, f["rho"], f["mu"], f["dt"],
                  "fibre", kappa, [Segment(X, False, ds)], random_rhs(N, seed))


def fibre_inflow_velocity(N: int, U: float = 1.0, noise: float = 0.1, seed: int = 0) -> np.ndarray:
    """Velocity u^n (2N^2: u block, then v block) at the start of a fibre step:
    the downward stream of Section 5.3, (0, -U), plus seeded uniform noise of
    amplitude noise * U per face from default_rng([seed, 5])."""
    u = np.zeros(2 * N * N)
    u[N * N:] = -U
    return u + noise * U * np.random.default_rng([seed, 5]).uniform(-1.0, 1.0, 2 * N * N)


# Configurations named after the workloads they describe.
def small_target(seed: int = 0) -> System:
    """32x32 grid, 3-level V-cycle, target points on a circle, kappa 1e4."""
    return target_circle(32, 3, 1e4, seed)


def membrane_256(kappa: float, seed: int = 0) -> System:
    return membrane_ellipse(256, None, kappa, seed)


def beam_512(kappa_b: float = 1.0, seed: int = 0) -> System:
    return beam_fibres(512, 5, kappa_b, 1e4, 4, 0.4, seed)


def batched_mix(n_systems: int = 64, seed0: int = 0, grids=(64, 128, 256, 512)) -> List[System]:
    """Independent systems: grid drawn from `grids`, law drawn uniformly from
    target / membrane / beam, stiffness log-uniform in [1e2, 1e6], coarsest
    grid 8x8. System s uses seed s (geometry stream default_rng([s, 2]))."""
    out = []
    for s in range(seed0, seed0 + n_systems):
        g = np.random.default_rng([s, 2])
        N = int(grids[g.integers(len(grids))])
        law = ("target", "membrane", "beam_open")[g.integers(3)]
        kappa = float(10.0 ** g.uniform(2.0, 6.0))
        L = levels_to(N, 8)
        if law == "target":
            sy = target_circle(N, L, kappa, s)
        elif law == "membrane":
            sy = membrane_ellipse(N, L, kappa, s)
        else:
            sy = beam_fibres(N, L, kappa_b=kappa, kappa_s=1e4, seed=s)
        out.append(sy)
    return out


# The paper's own context problems (Section 5), first backward-Euler step:
# dt = h/2, markers ~h/2 apart (membrane) or ~h apart (beam).
def paper_membrane(N: int, kappa: float = 1e4, mu: float = 1e-2, seed: int = 0) -> System:
    h = 1.0 / N
    seg = ellipse(0.5, 0.5, 0.23, 0.27, h / 2)
    return System(f"paper_membrane_N{N}", N, levels_to(N, 8), 1.0, mu, h / 2, "membrane",
                  {"kappa_s": kappa}, [seg], random_rhs(N, seed))


def paper_beam(N: int, kappa_b: float = 1.0, mu: float = 1e-2, seed: int = 0) -> System:
    h = 1.0 / N
    seg = trefoil_radius_curve(0.5, 0.5, 0.23, 0.035, h)
    return System(f"paper_beam_N{N}", N, levels_to(N, 8), 1.0, mu, h / 2, "beam_closed",
                  {"kappa_b": kappa_b}, [seg], random_rhs(N, seed))


def paper_target(N: int, kappa: float = 1e6, mu: float = 1.0, seed: int = 0) -> System:
    h = 1.0 / N
    segs = [row_of_markers(0.25, h / 2), row_of_markers(0.75, h / 2)]
    return System(f"paper_target_N{N}", N, levels_to(N, 8), 1.0, mu, h / 2, "target",
                  {"kappa_t": kappa}, segs, random_rhs(N, seed))


# ---------------------------------------------------------------------------
# learned correction stage: seeded initial weights and sample draws
# ---------------------------------------------------------------------------
NET_SHAPES = ((32, 3, 3, 3), (32, 32, 3, 3), (3, 32, 3, 3))


def net_init(seed: int = 0, out_scale: float = 1.0) -> np.ndarray:
    """Initial master weights (float32, 10 944): each layer uniform on
    [-s, s] with s = sqrt(6 / fan_in), fan_in = input channels x 9; the output
    layer is multiplied by out_scale (a small value starts training from a
    near-zero correction)."""
    rng = np.random.default_rng([seed, 3])
    parts = []
    for k, (co, ci, kh, kw) in enumerate(NET_SHAPES):
        s = math.sqrt(6.0 / (ci * kh * kw))
        parts.append(rng.uniform(-s, s, co * ci * kh * kw) * (out_scale if k == len(NET_SHAPES) - 1 else 1.0))
    return np.concatenate(parts).astype(np.float32)


def random_solutions(N: int, count: int, seed: int) -> np.ndarray:
    """count exact solutions x* (count x 3N^2): uniform[-1, 1] entries with the
    pressure block shifted to mean zero."""
    rng = np.random.default_rng([seed, 4])
    x = rng.uniform(-1.0, 1.0, (count, 3 * N * N))
    x[:, 2 * N * N:] -= x[:, 2 * N * N:].mean(axis=1, keepdims=True)
    return x


def batch_order(n_samples: int, batch: int, steps: int, seed: int = 0):
    """Sample indices for `steps` training batches: consecutive slices of
    fresh random permutations of range(n_samples) (one per epoch)."""
    rng = np.random.default_rng([seed, 5])
    perm = rng.permutation(n_samples)
    pos = 0
    for _ in range(steps):
        if pos + batch > n_samples:
            perm = rng.permutation(n_samples)
            pos = 0
        yield perm[pos:pos + batch].astype(np.int32)
        pos += batch
