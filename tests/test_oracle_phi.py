"""Pins of the phi_1 evaluations (paper Section 4).

* scalar phi_1 against its power series, its x = 0 value and its
  asymptote -1/x, and phi_2 against (phi_1 - 1)/x;
* the diagonalisation route against scipy's Pade expm of the augmented
  block matrix, and that block matrix against e^X = I + X phi_1(X).
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import operators as op
from oracle.phi import (expm_matrix, phi1_dense_expm, phi1_matrix, phi1_scalar,
                        phi2_scalar)


def _series(x, k0):
    """sum_i x^i / (i + k0)! by brute force (|x| <= 2), math.fsum."""
    return math.fsum(x**i / math.factorial(i + k0) for i in range(40))


def test_phi1_scalar_values():
    assert phi1_scalar(np.array([0.0]))[0] == 1.0
    for x in (-2.0, -0.3, -1e-6, 1e-9, 0.7, 2.0):
        assert abs(phi1_scalar(np.array([x]))[0] - _series(x, 1)) < 2e-16 * 4
        assert abs(phi2_scalar(np.array([x]))[0] - _series(x, 2)) < 2e-16 * 4
    big = np.array([-1e3, -1e6, -1e12])
    np.testing.assert_allclose(phi1_scalar(big), -1.0 / big, rtol=1e-15)
    np.testing.assert_allclose(phi2_scalar(big), 1.0 / big**2 * (-1.0 - big),
                               rtol=1e-15)


def test_augmented_block_identity():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((7, 7))
    P = phi1_dense_expm(X)
    np.testing.assert_allclose(np.eye(7) + X @ P, sla.expm(X), atol=1e-13)


@pytest.mark.parametrize("n", [5, 24])
@pytest.mark.parametrize("kind", ["rho2", "rho3", "phi", "z", "theta"])
@pytest.mark.parametrize("c", [1e-4, 1e-2, 0.5])
def test_phi1_matrix_diagonalisation_vs_pade(n, kind, c):
    A = {"rho2": op.A_rho(n, 2), "rho3": op.A_rho(n, 3), "phi": op.A_phi(n),
         "z": op.A_z(n), "theta": op.A_theta(n)}[kind]
    P = phi1_matrix(A, c)
    R = phi1_dense_expm(c * A)
    np.testing.assert_allclose(P, R, atol=5e-14 * n, rtol=0)
    np.testing.assert_allclose(expm_matrix(A, c), sla.expm(c * A), atol=5e-14 * n, rtol=0)
