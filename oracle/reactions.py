"""Reaction terms g(w) of the coupled systems (paper Section 5).

Each model maps a list of species fields to a list of reaction fields of
the same shape, evaluated pointwise at t_n (explicitly, eq. (BVAM_SExpE)).
"""
from __future__ import annotations

import math

import numpy as np


# --- Schnakenberg kinetics, eq. (schnaknl) with alpha_1 = 1 -----------------

def schnakenberg(U, a, b):
    u, v = U
    u2v = u * u * v
    return [a - u + u2v, b - u2v]


def schnakenberg_equilibrium(a, b):
    """Spatially uniform steady state (alpha_2 + beta_1, beta_1/(alpha_2+beta_1)^2)."""
    return [a + b, b / (a + b) ** 2]


def schnakenberg_jacobian(U, a, b):
    """J[r][s] = d g_r / d w_s, pointwise."""
    u, v = U
    return [[-1.0 + 2.0 * u * v, u * u], [-2.0 * u * v, -u * u]]


# --- Schnakenberg kinetics with the factor alpha_1, eqs. (schnaksys), (schnaknl)
# (Section 5.3): g = alpha_1 (b(u, v), c(u, v)); p = (alpha_2, beta_1, alpha_1).

def schnakenberg_scaled(U, a, b, gamma):
    return [gamma * g for g in schnakenberg(U, a, b)]


def schnakenberg_scaled_equilibrium(a, b, gamma):
    return schnakenberg_equilibrium(a, b)


def schnakenberg_scaled_jacobian(U, a, b, gamma):
    return [[gamma * x for x in row] for row in schnakenberg_jacobian(U, a, b)]


# --- BVAM kinetics, eq. (BVAMnl) ---------------------------------------------

BVAM_FIG1 = dict(gamma=3.87e-3, delta=7.5e-3, alpha1=8.99e-1, alpha2=2e-1,
                 alpha3=2e-1, beta1=-9.1e-1, beta2=-8.99e-1)


def bvam(U, alpha1, alpha2, alpha3, beta1, beta2):
    u, v = U
    bu = alpha1 * u * (1.0 - alpha2 * v * v) + v * (1.0 - alpha3 * u)
    cv = beta1 * v * (1.0 + alpha1 * alpha2 / beta1 * u * v) + u * (beta2 + alpha3 * v)
    return [bu, cv]


def bvam_exact(t, rho, theta):
    """Exact solution of the Section 5.1 test (u, v) on a (rho, theta) mesh."""
    f = np.exp(-t) * (1.0 - rho) ** 2
    return [f * np.exp(np.cos(theta) / 10.0), f * np.exp(np.sin(theta) / 10.0)]


def bvam_sources(t, rho, theta, p=BVAM_FIG1):
    """Manufactured sources b_s, c_s of Section 5.1.

    b_s = d_t u - gamma Lap_D u - b(u, v) with the *continuous* polar
    Laplacian (eq. (lapdisk)) of the exact solution, likewise c_s.
    For u = e^{-t} f(rho) g(theta): Lap_D u = e^{-t}[(f'/rho + f'') g + f g''/rho^2].
    """
    et = math.exp(-t)
    f = (1.0 - rho) ** 2
    f1 = -2.0 * (1.0 - rho)
    f2 = 2.0 * np.ones_like(rho)
    gu = np.exp(np.cos(theta) / 10.0)
    gu2 = (np.sin(theta) ** 2 / 100.0 - np.cos(theta) / 10.0) * gu
    gv = np.exp(np.sin(theta) / 10.0)
    gv2 = (np.cos(theta) ** 2 / 100.0 - np.sin(theta) / 10.0) * gv
    u = et * f * gu
    v = et * f * gv
    lap_u = et * ((f1 / rho + f2) * gu + f * gu2 / rho**2)
    lap_v = et * ((f1 / rho + f2) * gv + f * gv2 / rho**2)
    r = bvam([u, v], p["alpha1"], p["alpha2"], p["alpha3"], p["beta1"], p["beta2"])
    bs = -u - p["gamma"] * lap_u - r[0]
    cs = -v - p["delta"] * lap_v - r[1]
    return [bs, cs]


# --- 3-species activator / substrate / inhibitor (builder's model) ----------
# g_u = a - u + u^2 v - kappa u w,  g_v = b - u^2 v,  g_w = mu (u - w).
# Not from the paper: it is the reading adopted for the 3-species workload.

def ais3(U, a, b, kappa, mu):
    u, v, w = U
    u2v = u * u * v
    return [a - u + u2v - kappa * u * w, b - u2v, mu * (u - w)]


def ais3_equilibrium(a, b, kappa, mu):
    ue = (-1.0 + math.sqrt(1.0 + 4.0 * kappa * (a + b))) / (2.0 * kappa)
    return [ue, b / ue**2, ue]


def ais3_jacobian(U, a, b, kappa, mu):
    u, v, w = U
    one = np.ones_like(u)
    return [[-1.0 + 2.0 * u * v - kappa * w, u * u, -kappa * u],
            [-2.0 * u * v, -u * u, 0.0 * one],
            [mu * one, 0.0 * one, -mu * one]]


# --- DIB kinetics, eqs. (DIBnl) (Section 5.4) and (bulkcylnl) (Section 5.6) --
# Surface species (r, s); p = (zeta1, zeta2, zeta3, zeta4, zeta5, eta1, eta2,
# eta3, eta4, eta5).  g_r = zeta1 p(ub, r, s), g_s = zeta1 q(vb, r, s) with
#   p(u, r, s) = zeta2 u (1 - s) r - zeta3 r^3 - zeta4 (s - zeta5),
#   q(v, r, s) = eta1 v (1 + eta2 r)(1 - s)(1 - eta3 (1 - s))
#                - eta4 (1 + eta5 r) s (1 + eta3 s),
# where (ub, vb) are the bulk values below the surface point in the
# bulk-surface model of Section 5.6 and 1 in the surface-only model of
# Section 5.4 (whose p, q are the same with u = v = 1).

def dib_pq(ub, vb, r, s, zeta1, zeta2, zeta3, zeta4, zeta5, eta1, eta2, eta3, eta4, eta5):
    """(p, q) of eq. (bulkcylnl) (without the factor zeta1)."""
    pr = zeta2 * ub * (1.0 - s) * r - zeta3 * r**3 - zeta4 * (s - zeta5)
    qs = (eta1 * vb * (1.0 + eta2 * r) * (1.0 - s) * (1.0 - eta3 * (1.0 - s))
          - eta4 * (1.0 + eta5 * r) * s * (1.0 + eta3 * s))
    return pr, qs


def dib(U, *p):
    r, s = U
    pr, qs = dib_pq(1.0, 1.0, r, s, *p)
    return [p[0] * pr, p[0] * qs]


def dib_eta4(zeta5, eta1, eta3, beta2=1.0):
    """eta4 that makes (r, s) = (0, zeta5) an equilibrium when v = beta2
    (the formula after eq. (DIBnl), with beta2 = 1, and the one of Section
    5.6)."""
    return beta2 * eta1 * (1.0 - zeta5) * (1.0 - eta3 + eta3 * zeta5) / (zeta5 * (1.0 + eta3 * zeta5))


def dib_equilibrium(*p):
    return [0.0, p[4]]


def dib_jacobian(U, *p):
    r, s = U
    z1, z2, z3, z4, _, e1, e2, e3, e4, e5 = p
    one = np.ones_like(r)
    dp_dr = z2 * (1.0 - s) - 3.0 * z3 * r * r
    dp_ds = -z2 * r - z4 * one
    g = (1.0 - s) * (1.0 - e3 * (1.0 - s))  # d/ds of g: -(1 - e3 (1 - s)) + e3 (1 - s)
    dq_dr = e1 * e2 * g - e4 * e5 * s * (1.0 + e3 * s)
    dq_ds = (e1 * (1.0 + e2 * r) * (-(1.0 - e3 * (1.0 - s)) + e3 * (1.0 - s))
             - e4 * (1.0 + e5 * r) * (1.0 + 2.0 * e3 * s))
    return [[z1 * dp_dr, z1 * dp_ds], [z1 * dq_dr, z1 * dq_ds]]


# --- linear relaxation kinetics, eq. (bulkcylnl): g_s = -k_s (w_s - c_s) -----
# p = (k_0, c_0, k_1, c_1, ...): Section 5.6's b(u) = -alpha1 (u - alpha2),
# c(v) = -beta1 (v - beta2) with p = (alpha1, alpha2, beta1, beta2).

def linear(U, *p):
    return [-p[2 * s] * (U[s] - p[2 * s + 1]) for s in range(len(U))]


def linear_equilibrium(*p):
    return [p[2 * s + 1] for s in range(len(p) // 2)]


def linear_jacobian(U, *p):
    ns = len(U)
    one = np.ones_like(U[0])
    return [[(-p[2 * r] * one if r == s else 0.0 * one) for s in range(ns)] for r in range(ns)]


MODELS = {
    "schnakenberg": (schnakenberg, schnakenberg_equilibrium, schnakenberg_jacobian),
    "ais3": (ais3, ais3_equilibrium, ais3_jacobian),
    "schnakenberg_scaled": (schnakenberg_scaled, schnakenberg_scaled_equilibrium, schnakenberg_scaled_jacobian),
    "dib": (dib, dib_equilibrium, dib_jacobian),
    "linear": (linear, linear_equilibrium, linear_jacobian),
}


def reaction(kind, U, params):
    return MODELS[kind][0](U, *params)


def equilibrium(kind, params):
    return MODELS[kind][1](*params)


def jacobian(kind, U, params):
    return MODELS[kind][2](U, *params)
