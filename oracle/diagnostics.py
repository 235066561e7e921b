"""Indicators of a steady state (paper Section 5.2, the text after the disk
experiment): the integral mean of a species over the domain,

    (1 / |Omega|) * integral of u over Omega,

and the L2 norm of the increment of one time step,

    ( integral of (u(t_{n+1}) - u(t_n))^2 over Omega )^(1/2).

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this package.

The paper does not print the quadrature.  Reading taken here: each grid
point owns the cell between the midpoints to its neighbours along every
coordinate, the first and last cells closed by the ends of the coordinate's
range (rho in [0, rho_*], phi in [0, pi], z in [0, z_*]; theta cells have
width 2 pi / n), and its weight is the measure of that cell in the
geometry's volume element:

    disk, anomalous disk   rho drho dtheta
    sphere (radius rho_*)  rho_*^2 sin(phi) dtheta dphi
    ball                   rho^2 sin(phi) drho dtheta dphi
    cylinder               rho drho dtheta dz

so the weights sum to |Omega| exactly and the mean of a constant is that
constant.  The discrete mean is sum(w u) / sum(w).
"""
from __future__ import annotations

import math

import numpy as np

from . import operators as op


def cell_edges(points: np.ndarray, lo: float, hi: float) -> np.ndarray:
    """n + 1 cell boundaries: lo, the midpoints between neighbours, hi."""
    mid = 0.5 * (points[1:] + points[:-1])
    return np.concatenate([[lo], mid, [hi]])


def _rho_measure(points, rho_star, power):
    """integral of rho^power over each cell of [0, rho_*]."""
    e = cell_edges(points, 0.0, rho_star)
    return (e[1:] ** (power + 1) - e[:-1] ** (power + 1)) / (power + 1)


def _phi_measure(points):
    """integral of sin(phi) over each cell of [0, pi]."""
    e = cell_edges(points, 0.0, math.pi)
    return np.cos(e[:-1]) - np.cos(e[1:])


def _theta_measure(n):
    return np.full(n, 2.0 * math.pi / n)


def weights_1d(geometry: str, n, extent=(1.0, 1.0)):
    """Per-mode weight vectors (paper order); their outer product is the
    weight of each grid point."""
    rho_star, second = extent
    if geometry == "disk":
        return [_rho_measure(op.rho_grid(n[0], 2, rho_star), rho_star, 1), _theta_measure(n[1])]
    if geometry == "disk_lambda":
        return [_rho_measure(op.rho_lambda_grid(n[0], second, rho_star), rho_star, 1), _theta_measure(n[1])]
    if geometry == "sphere":
        return [rho_star**2 * _theta_measure(n[0]), _phi_measure(op.phi_grid(n[1]))]
    if geometry == "ball":
        return [_rho_measure(op.rho_grid(n[0], 3, rho_star), rho_star, 2), _theta_measure(n[1]),
                _phi_measure(op.phi_grid(n[2]))]
    if geometry == "cylinder":
        z = op.z_grid(n[2], second)
        ez = cell_edges(z, 0.0, second)
        return [_rho_measure(op.rho_grid(n[0], 2, rho_star), rho_star, 1), _theta_measure(n[1]),
                ez[1:] - ez[:-1]]
    raise ValueError(geometry)


def weights(geometry: str, n, extent=(1.0, 1.0)) -> np.ndarray:
    """Weight of every grid point, indexed [i, j(, k)] like the oracle's fields."""
    w = weights_1d(geometry, n, extent)
    out = w[0]
    for v in w[1:]:
        out = np.multiply.outer(out, v)
    return out


def integral_mean(U: np.ndarray, w: np.ndarray) -> float:
    return float(np.sum(w * U) / np.sum(w))


def increment_norm(U_new: np.ndarray, U_old: np.ndarray, w: np.ndarray) -> float:
    return float(math.sqrt(np.sum(w * (U_new - U_old) ** 2)))
