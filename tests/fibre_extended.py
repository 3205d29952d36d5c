"""Extended-precision force of the clamped flexible fibre (Section 5.3), for
pins of the double-precision forms: every coordinate and parameter is taken as
its exact binary value and the energies' gradient is evaluated with 60
significant digits (Python's decimal module), so rounding of the positions or
links cannot hide in the reference. Test helper, not collected."""
from decimal import Decimal, localcontext

import numpy as np


def straight_fibre_step(system, seed=3):
    """A nearly straight fibre on the workload's marker spacing (markers on the
    line y = 0.75 with a seeded 1e-6 ds jitter) and one step's displacement
    dt U for a smooth velocity of order one: the configuration in which the
    bending term's cross products lie far below the positions' rounding."""
    (seg,) = system.segments
    ds = seg.ds
    M = len(seg.X)
    m = int(system.kappa["m"])
    s = (np.arange(M) - m) * ds
    rng = np.random.default_rng(seed)
    Xn = np.stack([0.5 + s, 0.75 + 1e-6 * ds * rng.standard_normal(M)], axis=1).ravel()
    U = np.stack([0.05 * np.sin(7 * s), -1.0 + 1e-3 * np.cos(5 * s)], axis=1).ravel()
    return Xn, system.dt * U


def force(Xn, disp, p) -> np.ndarray:
    """F = -(1/ds) grad(E_b + E_s + E_p + E_t) at the exact positions Xn + disp,
    rounded to double at the end (interleaved 2M)."""
    with localcontext() as ctx:
        ctx.prec = 60
        M = len(Xn) // 2
        X = [(Decimal(Xn[2 * k]) + Decimal(disp[2 * k]), Decimal(Xn[2 * k + 1]) + Decimal(disp[2 * k + 1]))
             for k in range(M)]
        ds, EI, Ks = Decimal(p["ds"]), Decimal(p["EI"]), Decimal(p["K_s"])
        Kp, Kt, m = Decimal(p["K_p"]), Decimal(p["K_t"]), int(p["m"])
        D = [(X[k + 1][0] - X[k][0], X[k + 1][1] - X[k][1]) for k in range(M - 1)]
        G = [[Decimal(0), Decimal(0)] for _ in range(M)]
        wb = EI / ds ** 5
        for k in range(M - 2):              # bending, (EI / 2 ds^5) (D_k x D_{k+1})^2
            a, b = D[k], D[k + 1]
            c = wb * (a[0] * b[1] - a[1] * b[0])
            dca, dcb = (b[1], -b[0]), (-a[1], a[0])
            for t in range(2):
                G[k][t] -= c * dca[t]
                G[k + 1][t] += c * (dca[t] - dcb[t])
                G[k + 2][t] += c * dcb[t]
        for k in range(M - 1):              # stretching, (K_s / 2 ds) (|D_k| - ds)^2
            d = D[k]
            L = (d[0] * d[0] + d[1] * d[1]).sqrt()
            f = Ks / ds * (L - ds) / L
            for t in range(2):
                G[k][t] -= f * d[t]
                G[k + 1][t] += f * d[t]
        Xc = (Decimal(float(p["Xc"][0])), Decimal(float(p["Xc"][1])))
        for t in range(2):                  # position penalty
            G[m][t] += Kp * (X[m][t] - Xc[t])
        g = ((X[m + 1][0] - X[m - 1][0]) / (2 * ds) - 1, (X[m + 1][1] - X[m - 1][1]) / (2 * ds))
        for t in range(2):                  # tangent penalty
            G[m + 1][t] += Kt * g[t] / (2 * ds)
            G[m - 1][t] -= Kt * g[t] / (2 * ds)
        return np.array([float(-G[k][t] / ds) for k in range(M) for t in range(2)])
