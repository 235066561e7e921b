"""phi functions (paper Section 4).

phi_1(X) = sum_i X^i / (i+1)! ;  scalar phi_1(x) = (e^x - 1)/x, phi_1(0) = 1.
The scalar form is evaluated with expm1 so that small |x| does not cancel.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .operators import symmetriser


def phi1_scalar(x):
    """Elementwise phi_1 with phi_1(0) = 1 exactly."""
    x = np.asarray(x, dtype=float)
    out = np.ones_like(x)
    nz = x != 0.0
    out[nz] = np.expm1(x[nz]) / x[nz]
    return out


def phi2_scalar(x):
    """phi_2(x) = (e^x - 1 - x)/x^2 = (phi_1(x) - 1)/x, phi_2(0) = 1/2.

    For |x| < 1e-3 the Taylor series 1/2 + x/6 + x^2/24 + x^3/120 is used
    (truncation below 1e-14 there), avoiding the cancellation in (phi_1-1)/x.
    """
    x = np.asarray(x, dtype=float)
    out = np.empty_like(x)
    small = np.abs(x) < 1e-3
    xs = x[small]
    out[small] = 0.5 + xs / 6.0 + xs**2 / 24.0 + xs**3 / 120.0
    xl = x[~small]
    out[~small] = (np.expm1(xl) - xl) / xl**2
    return out


def eig_tridiag(A: np.ndarray):
    """Real eigen-decomposition A = V diag(lam) V^{-1} through the symmetriser.

    Proposition 1: A Xi = Xi S with S symmetric, S = Q Lambda Q^T, so
    V = Xi Q and V^{-1} = Q^T Xi^{-1}.  For a symmetric A (A_theta) Xi = I.
    """
    if np.allclose(A, A.T, rtol=0, atol=0):
        lam, Q = np.linalg.eigh(A)
        _exact_zero_eigenvalue(A, lam)
        return lam, Q, Q.T.copy()
    xi = symmetriser(A)
    S = (A * xi[None, :]) / xi[:, None]  # Xi^{-1} A Xi
    S = 0.5 * (S + S.T)  # exact symmetry up to rounding of the products above
    lam, Q = np.linalg.eigh(S)
    _exact_zero_eigenvalue(A, lam)
    V = xi[:, None] * Q
    Vinv = Q.T / xi[None, :]
    return lam, V, Vinv


def _exact_zero_eigenvalue(A, lam):
    """Operators with zero row sums (Neumann, periodic and pole-free ends)
    have the constants as an eigenvector with eigenvalue exactly 0, the case
    the scalar phi_1(0) = 1 of Section 4 is written for.  The eigensolver
    returns it only to O(eps ||A||); that residue, multiplied by tau d and
    by 1/rho^2 or 1/sin^2 scalings, would perturb the constant mode, so the
    eigenvalue closest to 0 is set to 0 exactly."""
    scale = np.abs(A).max()
    if np.abs(A.sum(axis=1)).max() <= 1e-12 * scale:
        k = int(np.argmin(np.abs(lam)))
        assert abs(lam[k]) <= 1e-10 * scale
        lam[k] = 0.0


def phi1_matrix(A: np.ndarray, c: float) -> np.ndarray:
    """phi_1(c A) for a 1D operator A by diagonalisation (Section 4)."""
    lam, V, Vinv = eig_tridiag(A)
    return (V * phi1_scalar(c * lam)[None, :]) @ Vinv


def expm_matrix(A: np.ndarray, c: float) -> np.ndarray:
    lam, V, Vinv = eig_tridiag(A)
    return (V * np.exp(c * lam)[None, :]) @ Vinv


def phi1_dense_expm(X) -> np.ndarray:
    """phi_1(X) as the top-right block of exp([[X, I], [0, 0]]) (tiny X only).

    Exponentiating the block matrix gives [[e^X, phi_1(X)], [0, I]] because
    the top-right block sums X^i/(i+1)!; scipy's expm is an independent
    (Pade scaling-and-squaring) route used to pin the eigen route.
    """
    X = np.asarray(X.toarray() if hasattr(X, "toarray") else X, dtype=float)
    n = X.shape[0]
    B = np.zeros((2 * n, 2 * n))
    B[:n, :n] = X
    B[:n, n:] = np.eye(n)
    return sla.expm(B)[:n, n:]
