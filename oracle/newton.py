"""One backward-Euler IB step with the flexible-fibre force, by Newton's method
(Section 2 scheme, Section 5.3) — test infrastructure.

The semi-implicit scheme of Section 2 evaluates interpolation and spreading at
the start of the step (J^n = J[X^n], S^n = S[X^n]) and the force at the new
configuration X^{n+1} = X^n + dt J^n u^{n+1}. With the explicit terms folded
into rhs, the unknowns x = (u, p) solve R(x) = 0,

    R(x) = K_0 x - [S^n F(X^n + dt J^n u); 0] - rhs,

K_0 = [[A_0, G], [-D, 0]] the Stokes part of Eq. intro_saddle. Its Jacobian
is K_E with A = A_0 - dt S^n E J^n and E = DF at the current configuration
(Section 2: the tangent of a nonlinear law replaces E). Newton's method takes
x <- x + dx with K_E dx = -R(x) until ||R|| <= rtol ||R_0|| or ||R|| <= atol
(Section 5.3). Here every Newton system is solved directly (oracle.direct,
mean-zero pressure), so the iterates are those of exact Newton. The force and
its tangent see the links of X^n updated by the displacement's differences
(Section 5.3), not differences of the absolute positions.
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np
import scipy.sparse as sp

from . import direct, fibre, ib, mac


def fibre_params(system) -> dict:
    """Parameters of oracle.fibre from a fibre-law system's kappa."""
    (seg,) = system.segments
    k = system.kappa
    return dict(ds=seg.ds, EI=k["EI"], K_s=k["K_s"], K_p=k["K_p"], K_t=k["K_t"], m=int(k["m"]),
                Xc=np.array([k["clamp_x"], k["clamp_y"]]))


class Step:
    """The pieces of one step at X^n: J^n, S^n, K_0 and the residual."""

    def __init__(self, system):
        self.s = system
        self.N = system.N
        self.n2 = system.N * system.N
        self.Xn = np.asarray(system.markers(), dtype=np.float64).ravel()
        self.p = fibre_params(system)
        self.J = ib.interpolation(system.N, system.markers())
        self.S = ib.spreading(system.N, self.J, system.weights())
        self.K0 = mac.reduced_operator(system.N, system.rho, system.mu, system.dt,
                                       sp.csr_matrix((2 * self.n2, 2 * self.n2)))

    def displacement(self, x) -> np.ndarray:
        """dt J^n u (interleaved)."""
        return self.s.dt * (self.J @ x[:2 * self.n2])

    def configuration(self, x) -> np.ndarray:
        """X^n + dt J^n u (interleaved)."""
        return self.Xn + self.displacement(x)

    def links(self, x) -> np.ndarray:
        """Links of the configuration, updated incrementally from those of X^n
        (Section 5.3): D_k = D^n_k + (disp_{k+1} - disp_k)."""
        Xn = self.Xn.reshape(-1, 2)
        d = self.displacement(x).reshape(-1, 2)
        return (Xn[1:] - Xn[:-1]) + (d[1:] - d[:-1])

    def residual(self, x, rhs) -> np.ndarray:
        F = fibre.force(self.configuration(x), self.p, D=self.links(x))
        SF = np.concatenate([self.S @ F, np.zeros(self.n2)])
        return self.K0 @ x - SF - rhs

    def jacobian(self, x) -> sp.csr_matrix:
        E = fibre.tangent(self.configuration(x), self.p, D=self.links(x))
        return mac.reduced_operator(self.N, self.s.rho, self.s.mu, self.s.dt, (self.S @ E @ self.J).tocsr())


@dataclasses.dataclass
class NewtonResult:
    x: np.ndarray
    X: np.ndarray              # X^{n+1} at the solution
    corrections: int
    converged: bool
    residuals: List[float]     # ||R|| at every iterate, the initial one first


def solve(system, rhs, x0=None, rtol=1e-8, atol=1e-8, max_newton=20) -> NewtonResult:
    st = Step(system)
    x = np.zeros(3 * st.n2) if x0 is None else np.array(x0, dtype=np.float64)
    res = []
    k = 0
    while True:
        R = st.residual(x, rhs)
        rn = float(np.linalg.norm(R))
        res.append(rn)
        if rn <= rtol * res[0] or rn <= atol:
            return NewtonResult(x, st.configuration(x), k, True, res)
        if k == max_newton:
            return NewtonResult(x, st.configuration(x), k, False, res)
        x = x + direct.solve(st.jacobian(x), st.N, -R)
        k += 1
