"""Pins of the steady-state indicators (paper Section 5.2): the integral
mean and the L2 norm of a step's increment, with cell-measure weights.

* the weights sum to |Omega| in closed form for every geometry and extent;
* a constant's mean is the constant, and a constant shift c has increment
  |c| sqrt(|Omega|);
* means and norms of smooth functions converge at second order to their
  exact integrals over the continuous domain.
"""
import math

import numpy as np
import pytest

from oracle import diagnostics as D
from oracle import operators as op

AREA = {
    "disk": lambda e: math.pi * e[0] ** 2,
    "disk_lambda": lambda e: math.pi * e[0] ** 2,
    "sphere": lambda e: 4.0 * math.pi * e[0] ** 2,
    "ball": lambda e: 4.0 / 3.0 * math.pi * e[0] ** 3,
    "cylinder": lambda e: math.pi * e[0] ** 2 * e[1],
}
CASES = [("disk", (7, 12), (1.3, 1.0)), ("disk_lambda", (9, 8), (1.0, -1.95)),
         ("disk_lambda", (6, 5), (0.7, 0.5)), ("sphere", (10, 9), (1.7, 1.0)),
         ("ball", (8, 6, 11), (0.8, 1.0)), ("cylinder", (9, 10, 7), (1.2, 2.5)),
         ("ball", (3, 3, 3), (1.0, 1.0))]


def _grids(geometry, n, extent):
    if geometry == "disk_lambda":
        return [op.rho_lambda_grid(n[0], extent[1], extent[0]), op.theta_grid(n[1])]
    if geometry == "disk":
        return [op.rho_grid(n[0], 2, extent[0]), op.theta_grid(n[1])]
    if geometry == "sphere":
        return [op.theta_grid(n[0]), op.phi_grid(n[1])]
    if geometry == "ball":
        return [op.rho_grid(n[0], 3, extent[0]), op.theta_grid(n[1]), op.phi_grid(n[2])]
    return [op.rho_grid(n[0], 2, extent[0]), op.theta_grid(n[1]), op.z_grid(n[2], extent[1])]


@pytest.mark.parametrize("geometry,n,extent", CASES)
def test_weights_sum_to_the_measure(geometry, n, extent):
    w = D.weights(geometry, n, extent)
    assert w.shape == tuple(n) and (w > 0).all()
    assert abs(w.sum() - AREA[geometry](extent)) < 1e-13 * AREA[geometry](extent)


@pytest.mark.parametrize("geometry,n,extent", CASES)
def test_constants(geometry, n, extent):
    w = D.weights(geometry, n, extent)
    U = np.full(n, 0.37)
    assert abs(D.integral_mean(U, w) - 0.37) < 1e-15
    assert abs(D.increment_norm(U + 2.5, U, w) - 2.5 * math.sqrt(AREA[geometry](extent))) < 1e-12


def _field(geometry, n, extent, f):
    g = np.meshgrid(*_grids(geometry, n, extent), indexing="ij")
    return f(*g)


# (geometry, extent, function of the paper coordinates, exact mean, exact L2 norm^2)
SMOOTH = [
    ("disk", (1.3, 1.0), lambda r, t: r**2 * np.cos(t) ** 2, 1.3**2 / 4, math.pi * 1.3**6 * 3 / 6 / 4),
    ("disk_lambda", (1.0, -1.95), lambda r, t: r**2, 0.5, math.pi / 3),
    ("disk_lambda", (1.0, 0.5), lambda r, t: r**2, 0.5, math.pi / 3),
    ("sphere", (1.7, 1.0), lambda t, p: np.cos(p) ** 2, 1.0 / 3.0, 1.7**2 * 4 * math.pi / 5),
    ("ball", (0.8, 1.0), lambda r, t, p: r**2, 0.6 * 0.8**2, 4 * math.pi * 0.8**7 / 7),
    ("cylinder", (1.2, 2.5), lambda r, t, z: z**2 * r, None, None),
]


@pytest.mark.parametrize("geometry,extent,f,mean,norm2", SMOOTH)
def test_second_order_convergence(geometry, extent, f, mean, norm2):
    if geometry == "cylinder":
        # mean of r z^2 over the cylinder: (2/3 rho_*) (z_*^2 / 3); norm^2 = 2 pi rho_*^4/4 z_*^5/5
        mean = 2.0 / 3.0 * extent[0] * extent[1] ** 2 / 3.0
        norm2 = 2 * math.pi * extent[0] ** 4 / 4 * extent[1] ** 5 / 5
    errs = []
    for k in (1, 2, 4):
        n = {"disk": (16 * k, 24 * k), "disk_lambda": (16 * k, 8 * k), "sphere": (12 * k, 16 * k),
             "ball": (16 * k, 8 * k, 16 * k), "cylinder": (12 * k, 8 * k, 12 * k)}[geometry]
        w = D.weights(geometry, n, extent)
        U = _field(geometry, n, extent, f)
        em = abs(D.integral_mean(U, w) - mean) / abs(mean)
        en = abs(D.increment_norm(U, 0.0 * U, w) ** 2 - norm2) / norm2
        errs.append(max(em, en))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.0 < r1 < 5.5 and 3.0 < r2 < 5.5, errs
