"""Pins of the oracle's grids and 1D operators (paper Section 3, App. A).

Each check comes from mathematics the paper states or implies, not from
re-typing the stencil formulas: zero row sums (constants are harmonic),
second-order consistency on smooth functions satisfying the boundary
conditions, closed-form spectra, Proposition 1 and the sigma bounds of
Appendix A.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import operators as op
from oracle.phi import eig_tridiag

NS = [6, 17, 64]


@pytest.mark.parametrize("n", NS)
def test_row_sums(n):
    for A in (op.A_theta(n), op.A_rho(n, 2), op.A_rho(n, 3), op.A_phi(n)):
        scale = np.abs(A).max()
        assert np.abs(A @ np.ones(n)).max() <= 1e-13 * scale
    # Dirichlet end at z_*: A_z 1 = -e_n / h^2
    Az = op.A_z(n, 2.0)
    np.testing.assert_allclose(Az @ np.ones(n) + op.z_boundary_column(n, 2.0), 0.0,
                               atol=1e-13 * np.abs(Az).max())


def _consistency_error(n, which):
    """max |A f - L f| over all rows for a smooth f meeting the BCs."""
    if which == "rho2":
        r = op.rho_grid(n, 2)
        f = np.cos(math.pi * r)
        Lf = -math.pi * np.sin(math.pi * r) / r - math.pi**2 * np.cos(math.pi * r)
        return np.abs(op.A_rho(n, 2) @ f - Lf).max()
    if which == "rho3":
        r = op.rho_grid(n, 3)
        f = np.cos(math.pi * r)
        Lf = -2 * math.pi * np.sin(math.pi * r) / r - math.pi**2 * np.cos(math.pi * r)
        return np.abs(op.A_rho(n, 3) @ f - Lf).max()
    if which == "phi":  # Legendre P_1 = cos(phi) is an eigenfunction, eigenvalue -2
        p = op.phi_grid(n)
        return np.abs(op.A_phi(n) @ np.cos(p) + 2 * np.cos(p)).max()
    if which == "z":  # cos(pi z / 2): Neumann at 0, zero at z_* = 1
        z = op.z_grid(n, 1.0)
        f = np.cos(0.5 * math.pi * z)
        return np.abs(op.A_z(n, 1.0) @ f + (0.5 * math.pi) ** 2 * f).max()
    if which == "theta":
        t = op.theta_grid(n)
        return np.abs(op.A_theta(n) @ np.cos(2 * t) + 4 * np.cos(2 * t)).max()
    raise ValueError(which)


@pytest.mark.parametrize("which", ["rho2", "rho3", "phi", "z", "theta"])
def test_second_order_consistency(which):
    e1 = _consistency_error(40, which)
    e2 = _consistency_error(80, which)
    e3 = _consistency_error(160, which)
    # halving h divides the truncation error by ~4 (second order)
    assert 3.4 < e1 / e2 < 4.6 and 3.4 < e2 / e3 < 4.6, (e1, e2, e3)
    assert e3 < 5e-3


@pytest.mark.parametrize("n", [5, 16, 33])
def test_theta_closed_form_spectrum(n):
    h = 2 * math.pi / n
    lam = np.sort(-4.0 / h**2 * np.sin(math.pi * np.arange(n) / n) ** 2)
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(op.A_theta(n))), lam,
                               atol=1e-12 / h**2)


@pytest.mark.parametrize("n", [5, 16, 33])
def test_z_closed_form_eigenpairs(n):
    """Eigenpairs printed after eq. (A_z)."""
    zs = 1.3
    h = zs / n
    A = op.A_z(n, zs)
    for k in range(1, n + 1):
        a = math.pi * (k - 0.5) / n
        lam = -2 / h**2 + 2 / h**2 * math.cos(a)
        i = np.arange(1, n)
        v = np.append(np.sin((n - i + 1) * a) / math.sin(a), 1.0)
        np.testing.assert_allclose(A @ v, lam * v, atol=1e-11 * np.abs(v).max() / h**2)


@pytest.mark.parametrize("n", [6, 20, 50])
@pytest.mark.parametrize("kind", ["rho2", "rho3", "phi", "z", "theta"])
def test_proposition_1(n, kind):
    A = {"rho2": op.A_rho(n, 2), "rho3": op.A_rho(n, 3), "phi": op.A_phi(n),
         "z": op.A_z(n), "theta": op.A_theta(n)}[kind]
    off = A - np.diag(np.diag(A))
    assert (off[np.abs(off) > 0] > 0).all()  # 1. positive extra-diagonal entries
    sub = np.diag(A, -1)
    assert (sub > 0).all() and (np.diag(A, 1) > 0).all()
    scale = np.abs(A).max()
    for t in (0.01 / scale, 1.0 / scale, 10.0 / scale):
        assert sla.expm(t * A).min() >= -1e-14  # 2. nonnegative exponential
    ev = np.linalg.eigvals(A)
    assert np.abs(ev.imag).max() <= 1e-9 * scale  # real spectrum (3.)
    assert ev.real.max() <= 1e-10 * scale  # 5. nonpositive eigenvalues
    if kind != "theta":
        xi = op.symmetriser(A)
        S = (A * xi[None, :]) / xi[:, None]
        np.testing.assert_allclose(S, S.T, atol=1e-12 * scale)  # 3. A Xi = Xi S
    lam, V, Vinv = eig_tridiag(A)  # 4. diagonalisable, A V = V Lambda
    np.testing.assert_allclose(A @ V, V * lam[None, :], atol=1e-10 * scale)
    np.testing.assert_allclose(V @ Vinv, np.eye(n), atol=1e-11)


@pytest.mark.parametrize("n", [5, 12, 40, 101])
def test_symmetriser_norms(n):
    """||Xi||_2 = 1, ||Xi^-1||_2 = sqrt(2n-3) (d=2) and n-1 (d=3) (Prop. 1 proof)."""
    for d, target in ((2, math.sqrt(2 * n - 3)), (3, n - 1.0)):
        xi = op.symmetriser(op.A_rho(n, d))
        assert abs(xi.max() - 1.0) < 1e-14
        assert abs(1.0 / xi.min() - target) < 1e-10 * target


@pytest.mark.parametrize("n", [3, 8, 64, 128, 512, 2049])
def test_sigma_appendix_a(n):
    s = op.sigma_phi(n)
    assert 0.0 < s < 0.5
    assert s > (-(n - 1) + math.sqrt(n * n - 1.0)) / 2.0  # lower bound of App. A
    h = math.pi / (n - 1 + 2 * s)
    # both equations of system (syscn)
    assert abs(h - (math.pi - 2 * s * h) / (n - 1)) < 1e-15
    assert abs(-1.0 / math.tan(s * h) / (2 * h) + 1.0 / h**2) < 1e-13 / h**2


def test_sigma_tends_to_half():
    vals = [0.5 - op.sigma_phi(n) for n in (8, 64, 512, 4096)]
    assert all(a > b > 0 for a, b in zip(vals, vals[1:]))


@pytest.mark.parametrize("n", [7, 30])
def test_phi_grid_symmetric(n):
    p = op.phi_grid(n)
    np.testing.assert_allclose(p + p[::-1], math.pi, atol=1e-14)
    assert p[0] > 0 and p[-1] < math.pi
