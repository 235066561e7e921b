"""Grids and one-dimensional finite-difference operators (paper Section 3).

Every matrix is returned dense (n <= a few hundred) in float64.  The
tridiagonal convention is that of eq. (tridiag): row l holds
``[c_{l-1}, a_l, b_l]``, i.e. ``A[l, l+1] = b_l`` and ``A[l+1, l] = c_l``.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq


def tridiag(a, b, c) -> np.ndarray:
    """Dense matrix of eq. (tridiag) from diagonal a (n), super b (n-1), sub c (n-1)."""
    a = np.asarray(a, float)
    n = a.size
    A = np.diag(a)
    A[np.arange(n - 1), np.arange(1, n)] = b
    A[np.arange(1, n), np.arange(n - 1)] = c
    return A


# --- theta: periodic second derivative, eq. (A_theta) -----------------------

def theta_grid(n: int) -> np.ndarray:
    """theta_j = j h_theta, j = 1..n, h_theta = 2 pi / n."""
    h = 2.0 * math.pi / n
    return h * np.arange(1, n + 1)


def A_theta(n: int) -> np.ndarray:
    """Symmetric circulant [-2, 1, ..., 1] / h_theta^2, eq. (A_theta)."""
    h = 2.0 * math.pi / n
    A = -2.0 * np.eye(n) + np.eye(n, k=1) + np.eye(n, k=-1)
    A[0, n - 1] += 1.0
    A[n - 1, 0] += 1.0
    return A / h**2


# --- rho: radial operators, eqs. (disk_discr) and (ball_discr) --------------

def rho_grid(n: int, d: int, rho_star: float = 1.0) -> np.ndarray:
    """Half-point grid (d = 2) or rho_i = i h (d = 3)."""
    if d == 2:
        h = rho_star / (n - 0.5)
        return 0.5 * h + h * np.arange(n)
    if d == 3:
        h = rho_star / n
        return h * np.arange(1, n + 1)
    raise ValueError("d must be 2 or 3")


def A_rho(n: int, d: int, rho_star: float = 1.0) -> np.ndarray:
    """A_{rho,d}: (d-1)/rho d/drho + d^2/drho^2, Neumann at rho_* (Table 1)."""
    ell = np.arange(1, n)  # l = 1..n-1
    if d == 2:
        h = rho_star / (n - 0.5)
        b = 2.0 * ell / ((2.0 * ell - 1.0) * h**2)
        c = 2.0 * ell / ((2.0 * ell + 1.0) * h**2)
    elif d == 3:
        h = rho_star / n
        b = (ell + 1.0) / (ell * h**2)
        c = ell / ((ell + 1.0) * h**2)
    else:
        raise ValueError("d must be 2 or 3")
    c[-1] = 2.0 / h**2  # c_{n-1}: homogeneous Neumann row at rho_*
    a = np.full(n, -2.0 / h**2)
    return tridiag(a, b, c)


# --- rho of the anomalous operator Delta_lambda, eq. (A_lambda), Section 5.3 --
# Delta_lambda = (1 - lambda) rho^-(1+lambda) d/drho + rho^-lambda d^2/drho^2
# (+ rho^-(2+lambda) d^2/dtheta^2), homogeneous Dirichlet data at rho_* after
# lifting.  lambda = 0 is the polar Laplacian on the Dirichlet grid.

def rho_lambda_grid(n: int, lam: float, rho_star: float = 1.0) -> np.ndarray:
    """rho_i = (1 - lambda) h / 2 + (i - 1) h, h = rho_* / (n + (1 - lambda) / 2)."""
    s = 0.5 * (1.0 - lam)
    h = rho_star / (n + s)
    return s * h + h * np.arange(n)


def A_rho_lambda(n: int, lam: float, rho_star: float = 1.0) -> np.ndarray:
    """Tridiagonal A_lambda of eq. (A_lambda) in the layout of eq. (tridiag)
    (a diagonal, b super-, c sub-diagonal)."""
    s = 0.5 * (1.0 - lam)
    h = rho_star / (n + s)
    hp = h ** (2.0 + lam)
    ell = np.arange(1, n + 1, dtype=float)
    a = -2.0 / ((s + ell - 1.0) ** lam * hp)
    l = np.arange(1, n, dtype=float)
    b = (1.0 - lam + l - 1.0) / ((s + l - 1.0) ** (1.0 + lam) * hp)
    c = l / ((s + l) ** (1.0 + lam) * hp)
    return tridiag(a, b, c)


def rho_lambda_boundary(n: int, lam: float, rho_star: float = 1.0) -> float:
    """b_n: the coefficient of the Dirichlet value at rho_* in the last row."""
    s = 0.5 * (1.0 - lam)
    h = rho_star / (n + s)
    return (1.0 - lam + n - 1.0) / ((s + n - 1.0) ** (1.0 + lam) * h ** (2.0 + lam))


# --- phi: polar angle on (0, pi), eqs. (syscn), (A_phi), Appendix A ---------

def sigma_phi(n: int) -> float:
    """Root in (0, 1/2) of f(x) = cot(x pi / (n-1+2x)) - 2 (n-1+2x) / pi.

    Appendix A shows f is strictly decreasing with a sign change on (0, 1/2);
    the root is bracketed and driven to full double precision.
    """
    def f(x):
        return 1.0 / math.tan(x * math.pi / (n - 1 + 2 * x)) - 2.0 * (n - 1 + 2 * x) / math.pi

    return brentq(f, 1e-12, 0.5, xtol=1e-300, rtol=4 * np.finfo(float).eps, maxiter=500)


def phi_grid(n: int) -> np.ndarray:
    """phi_k = sigma h_phi + (k-1) h_phi, h_phi = pi / (n - 1 + 2 sigma)."""
    s = sigma_phi(n)
    h = math.pi / (n - 1 + 2 * s)
    return (s + np.arange(n)) * h


def A_phi(n: int) -> np.ndarray:
    """cot(phi) d/dphi + d^2/dphi^2 on the sigma-shifted grid, eq. (A_phi)."""
    s = sigma_phi(n)
    h = math.pi / (n - 1 + 2 * s)
    ell = np.arange(1, n)
    b = 1.0 / h**2 + 1.0 / np.tan((s + ell - 1) * h) / (2.0 * h)
    c = b[::-1].copy()  # c_l = b_{n-l}
    return tridiag(np.full(n, -2.0 / h**2), b, c)


# --- z: Neumann at 0, Dirichlet at z_*, eq. (A_z) --------------------------

def z_grid(n: int, z_star: float = 1.0) -> np.ndarray:
    h = z_star / n
    return h * np.arange(n)


def A_z(n: int, z_star: float = 1.0) -> np.ndarray:
    h = z_star / n
    b = np.full(n - 1, 1.0 / h**2)
    b[0] = 2.0 / h**2
    c = np.full(n - 1, 1.0 / h**2)
    return tridiag(np.full(n, -2.0 / h**2), b, c)


def z_boundary_column(n: int, z_star: float = 1.0) -> np.ndarray:
    """Coefficient of the Dirichlet value at z_* in each row (e_n / h_z^2)."""
    e = np.zeros(n)
    e[-1] = 1.0 / (z_star / n) ** 2
    return e


# --- Proposition 1: diagonal symmetriser ------------------------------------

def symmetriser(A: np.ndarray) -> np.ndarray:
    """Diagonal of Xi with xi_1 = 1, xi_{l+1} = sqrt(c_1..c_l / (b_1..b_l)).

    Then A Xi = Xi S with S symmetric (Proposition 1).
    """
    b = np.diag(A, 1)
    c = np.diag(A, -1)
    xi = np.ones(A.shape[0])
    xi[1:] = np.sqrt(np.cumprod(c / b))
    return xi


def operators_1d(geometry: str, n, extent=(1.0, 1.0)):
    """Per-mode dense 1D operators and grids for a geometry (paper order).

    ``extent`` = (rho_*, z_*); for "disk_lambda" (the anomalous operator of
    Section 5.3) the second entry is lambda.
    """
    rho_star, z_star = extent
    if geometry == "disk_lambda":
        nr, nt = n
        return {"A": [A_rho_lambda(nr, z_star, rho_star), A_theta(nt)],
                "grid": [rho_lambda_grid(nr, z_star, rho_star), theta_grid(nt)]}
    if geometry == "disk":
        nr, nt = n
        return {"A": [A_rho(nr, 2, rho_star), A_theta(nt)],
                "grid": [rho_grid(nr, 2, rho_star), theta_grid(nt)]}
    if geometry == "sphere":
        nt, nphi = n
        return {"A": [A_theta(nt), A_phi(nphi)],
                "grid": [theta_grid(nt), phi_grid(nphi)]}
    if geometry == "ball":
        nr, nt, nphi = n
        return {"A": [A_rho(nr, 3, rho_star), A_theta(nt), A_phi(nphi)],
                "grid": [rho_grid(nr, 3, rho_star), theta_grid(nt), phi_grid(nphi)]}
    if geometry == "cylinder":
        nr, nt, nz = n
        return {"A": [A_rho(nr, 2, rho_star), A_theta(nt), A_z(nz, z_star)],
                "grid": [rho_grid(nr, 2, rho_star), theta_grid(nt), z_grid(nz, z_star)]}
    raise ValueError(geometry)
