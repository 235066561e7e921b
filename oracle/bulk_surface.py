"""Bulk-surface Schnakenberg system on the ball (paper Section 5.5, eqs.
(bulkballsys), (bulkballnl)): u, v diffuse in the ball with the Laplacian of
eq. (lapball), r, s on its surface with rho_*^-2 times the Laplace-Beltrami
operator of eq. (lapsphere), coupled through Robin conditions

    du/dn = zeta1 (zeta2 r - zeta3 u),   delta dv/dn = zeta1 (eta1 s - eta2 v),

and the surface kinetics p = b(r, s) - (zeta2 r - zeta3 u),
q = c(r, s) - (eta1 s - eta2 v), all times zeta1 (b, c Schnakenberg's).

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this package.

The paper omits the discretisation of the coupling.  Reading taken here:

* the sphere's (theta, phi) grid is the ball's angular grid, so surface
  point (j, k) sits above bulk point (n, j, k) with rho_n = rho_*;
* the Robin condition enters the ball's boundary row by the same ghost
  point that gives its Neumann row: u_{n+1} = u_{n-1} + 2 h du/drho, which
  adds (1 + h / rho_*)(2 / h) du/drho to that row of A_{rho,3}; for v the
  factor delta of the condition cancels the diffusion coefficient, so both
  species gain kappa * zeta1 * (flux) with kappa = 2 (1 + 1/n) / h;
* the coupling terms, like the kinetics, are evaluated at t_n and enter the
  step through F (they are part of g); the diffusion factors of both
  surfaces are the uncoupled ones, so the split step of each domain is the
  plain ball / sphere step of Section 4.
"""
from __future__ import annotations

import numpy as np

from . import reactions as R
from .splitee import SplitEE

# Section 5.5: alpha_1 = zeta_1 = 55, alpha_2 = 0.1, beta_1 = 0.9,
# zeta_2 = zeta_3 = 5/12, eta_1 = eta_2 = 5, delta = epsilon = 10
PARAMS = dict(alpha1=55.0, alpha2=0.1, beta1=0.9, zeta1=55.0, zeta2=5.0 / 12.0, zeta3=5.0 / 12.0,
              eta1=5.0, eta2=5.0, delta=10.0, epsilon=10.0)


def kappa(n_rho: int, rho_star: float = 1.0) -> float:
    """Coefficient of du/drho in the ball's boundary row (ghost point)."""
    h = rho_star / n_rho
    return (2.0 / h) * (1.0 + h / rho_star)


def equilibrium(p=PARAMS):
    ue, ve = R.schnakenberg_equilibrium(p["alpha2"], p["beta1"])
    return [ue, ve], [ue, ve]


class BulkSurface:
    """Split exponential Euler for the coupled system: one ball split step
    for (u, v) and one sphere split step for (r, s) per time step, with the
    kinetics and the coupling of both evaluated at t_n.

    ``kinetics=False`` keeps only the coupling terms (for the conservation
    pin); fields are [i, j, k] (ball) and [j, k] (surface) arrays.
    """

    def __init__(self, n, tau, p=PARAMS, kinetics=True):
        self.n, self.tau, self.p, self.kinetics = tuple(n), tau, dict(p), kinetics
        self.ball = SplitEE("ball", self.n, [1.0, p["delta"]], tau, (1.0, 1.0))
        self.surface = SplitEE("sphere", (self.n[1], self.n[2]), [1.0, p["epsilon"]], tau, (1.0, 1.0))
        self.kappa = kappa(self.n[0])

    def fluxes(self, U, S):
        """zeta2 r - zeta3 u and eta1 s - eta2 v at the surface points."""
        p = self.p
        ub, vb = U[0][-1], U[1][-1]
        return p["zeta2"] * S[0] - p["zeta3"] * ub, p["eta1"] * S[1] - p["eta2"] * vb

    def reactions(self, U, S):
        """Explicit terms of F: bulk kinetics plus the Robin source in the
        boundary layer; surface kinetics minus the exchange."""
        p = self.p
        f_u, f_v = self.fluxes(U, S)
        if self.kinetics:
            Gb = R.schnakenberg_scaled(U, p["alpha2"], p["beta1"], p["alpha1"])
            Gs = R.schnakenberg_scaled(S, p["alpha2"], p["beta1"], p["zeta1"])
        else:
            Gb = [np.zeros_like(U[0]), np.zeros_like(U[1])]
            Gs = [np.zeros_like(S[0]), np.zeros_like(S[1])]
        Gb[0] = Gb[0].copy()
        Gb[1] = Gb[1].copy()
        Gb[0][-1] += self.kappa * p["zeta1"] * f_u
        Gb[1][-1] += self.kappa * p["zeta1"] * f_v
        Gs = [Gs[0] - p["zeta1"] * f_u, Gs[1] - p["zeta1"] * f_v]
        return Gb, Gs

    def step(self, U, S):
        Gb, Gs = self.reactions(U, S)
        U1 = self.ball.step(U, lambda _: Gb)
        S1 = self.surface.step(S, lambda _: Gs)
        return U1, S1
