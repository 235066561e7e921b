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


# ---------------------------------------------------------------------------
# Bulk-surface DIB model on the cylinder (paper Section 5.6, eqs.
# (bulkcylsys), (bulkcylnl)): u, v in a cylinder of radius rho_* and height
# z_* with linear kinetics b(u) = -alpha1 (u - alpha2), c(v) = -beta1 (v -
# beta2), Dirichlet data (alpha2, beta2) on the top disk, homogeneous Neumann
# data on the lateral surface, and on the bottom disk Omega_B the flux
# conditions grad u . n = -zeta1 alpha3 p(u, r, s), grad v . n = -zeta1 beta3
# q(v, r, s); r, s diffuse on Omega_B (disk Laplacian, Neumann at its rim)
# with kinetics zeta1 p(u, r, s), zeta1 q(v, r, s) (p, q of eq. (bulkcylnl)).
#
# The paper does not print the discretisation.  Reading taken here (as for
# the ball, R20-style):
#
# * the disk's (rho, theta) grid is the cylinder's, so surface point (i, j)
#   lies at the bottom of bulk column (i, j), on the bulk point (i, j, 1)
#   with z_1 = 0;
# * the flux enters the bulk's z = 0 row through the ghost point that makes
#   A_z's Neumann row: with outward normal -e_z the condition reads
#   du/dz(0) = zeta1 alpha3 p, and u_0 = u_2 - 2 h_z du/dz(0) adds
#   -(2 / h_z) du/dz(0) to (A_z u)_1; the diffusion coefficient multiplies
#   it (d_u = 1, d_v = delta), so F_u gains -(2 / h_z) zeta1 alpha3 p and
#   F_v gains -delta (2 / h_z) zeta1 beta3 q on the layer z = 0;
# * the coupling terms and all kinetics are evaluated at t_n and enter F;
#   each domain then takes its plain split step (eq. (ee_cylinder) with the
#   lifted Dirichlet data, eq. (ee_disk)).
#
# With the trapezoid weights h_z (1/2, 1, ..., 1) in z and the left null
# vector of the disk operator in (rho, theta), the weighted sums satisfy
# exactly  sum w_B F_u + alpha3 sum w_D F_r = sum w_D (u_D - u_n) / h_z
# + sum w_B b(u)  (and delta beta3 for v, s): the exchange moves mass
# between the bulk and the surface without creating any (pinned).

DIB_CYL = dict(alpha1=1.0, alpha2=1.0, alpha3=0.1, beta1=1.0, beta2=1.0, beta3=0.1, delta=1.0,
               epsilon=20.0, zeta1=1.0, zeta2=10.0, zeta3=1.0, zeta4=30.0, zeta5=0.5,
               eta1=3.0, eta2=2.5, eta3=0.2, eta5=1.5)
DIB_CYL["eta4"] = R.dib_eta4(DIB_CYL["zeta5"], DIB_CYL["eta1"], DIB_CYL["eta3"], DIB_CYL["beta2"])


def dib_params(p=DIB_CYL):
    """(zeta1, ..., zeta5, eta1, ..., eta5) in the order of reactions.dib."""
    return tuple(p[k] for k in ("zeta1", "zeta2", "zeta3", "zeta4", "zeta5",
                                "eta1", "eta2", "eta3", "eta4", "eta5"))


def linear_params(p=DIB_CYL):
    """(alpha1, alpha2, beta1, beta2) in the order of reactions.linear."""
    return (p["alpha1"], p["alpha2"], p["beta1"], p["beta2"])


def cylinder_equilibrium(p=DIB_CYL):
    """(u_e, v_e), (r_e, s_e) = (alpha2, beta2), (0, zeta5)."""
    return [p["alpha2"], p["beta2"]], [0.0, p["zeta5"]]


class BulkSurfaceCylinder:
    """Split exponential Euler for the Section 5.6 system: per time step one
    cylinder split step for (u, v) and one disk split step for (r, s), with
    every explicit term evaluated at t_n.

    Fields are [i, j, k] (cylinder, k along z with z_1 = 0) and [i, j]
    (bottom disk).  ``kinetics=False`` drops the bulk kinetics b, c (the
    surface kinetics p, q are the exchange itself and stay).
    """

    def __init__(self, n, tau, extent=(15.0, 25.0), p=DIB_CYL, kinetics=True):
        self.n, self.tau, self.p, self.kinetics = tuple(n), tau, dict(p), kinetics
        self.extent = tuple(extent)
        self.bulk = SplitEE("cylinder", self.n, [1.0, p["delta"]], tau, self.extent)
        self.surface = SplitEE("disk", (self.n[0], self.n[1]), [1.0, p["epsilon"]], tau, (self.extent[0], 1.0))
        self.hz = self.extent[1] / self.n[2]

    def pq(self, U, S):
        """p(u, r, s) and q(v, r, s) at the surface points (u, v on z = 0)."""
        return R.dib_pq(U[0][:, :, 0], U[1][:, :, 0], S[0], S[1], *dib_params(self.p))

    def reactions(self, U, S):
        """Explicit terms of F: bulk kinetics plus the flux of the z = 0 row;
        surface kinetics zeta1 (p, q)."""
        p = self.p
        pr, qs = self.pq(U, S)
        if self.kinetics:
            Gb = R.linear(U, *linear_params(p))
        else:
            Gb = [np.zeros_like(U[0]), np.zeros_like(U[1])]
        Gb = [g.copy() for g in Gb]
        Gb[0][:, :, 0] += -(2.0 / self.hz) * 1.0 * p["zeta1"] * p["alpha3"] * pr
        Gb[1][:, :, 0] += -(2.0 / self.hz) * p["delta"] * p["zeta1"] * p["beta3"] * qs
        Gs = [p["zeta1"] * pr, p["zeta1"] * qs]
        return Gb, Gs

    def F(self, U, S):
        """The full right-hand sides d M W + g (with the lifted Dirichlet data)."""
        Gb, Gs = self.reactions(U, S)
        wd = [self.p["alpha2"], self.p["beta2"]]
        Fb = [self.bulk.apply_M(U[s], s, wd[s]) + Gb[s] for s in range(2)]
        Fs = [self.surface.apply_M(S[s], s) + Gs[s] for s in range(2)]
        return Fb, Fs

    def step(self, U, S):
        Gb, Gs = self.reactions(U, S)
        U1 = self.bulk.step(U, lambda _: Gb, w_dirichlet=[self.p["alpha2"], self.p["beta2"]])
        S1 = self.surface.step(S, lambda _: Gs)
        return U1, S1

    def step_deviation(self, dU, dS):
        """The same step on the deviations from the equilibrium: the
        equilibrium is a fixed point of the linear part (M takes constants
        to zero, and the lifted Dirichlet value equals the bulk equilibrium),
        so W_e + dW steps to W_e + (dW stepped with the kinetics evaluated
        at W_e + dW and homogeneous Dirichlet data).  Stepping full values,
        the FP64 rounding of M (W_e + dW) costs eps |W_e| ||tau d M||, which
        the deviation form does not."""
        ub, us = cylinder_equilibrium(self.p)
        Gb, Gs = self.reactions([ub[s] + dU[s] for s in range(2)], [us[s] + dS[s] for s in range(2)])
        dU1 = self.bulk.step(dU, lambda _: Gb, w_dirichlet=[0.0, 0.0])
        dS1 = self.surface.step(dS, lambda _: Gs)
        return dU1, dS1
