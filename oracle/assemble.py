"""Kronecker-sum discretisations M = M_1 + ... + M_d (paper Section 2).

Vectors follow the paper's ordering, first grid index fastest
(eqs. (disk)-(cylinder)), which is NumPy's Fortran order for an array
indexed ``W[i, j(, k)]``.  All matrices are scipy.sparse CSR in float64.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import operators as op


def _kron(*mats):
    out = sp.csr_matrix(mats[0])
    for m in mats[1:]:
        out = sp.kron(out, sp.csr_matrix(m), format="csr")
    return out


def terms(geometry: str, n, extent=(1.0, 1.0)):
    """The split terms [M_1, ..., M_d] in the order the paper writes them.

    disk:     M = I (x) A_{rho,2} + A_theta (x) D_rho                 eq. (disk)
    sphere:   M = D_phi (x) A_theta + A_phi (x) I                     eq. (sphere)
    ball:     M = I(x)I(x)A_{rho,3} + D_phi(x)A_theta(x)D_rho
                  + A_phi(x)I(x)D_rho                                  eq. (ball)
    cylinder: M = I(x)I(x)A_{rho,2} + I(x)A_theta(x)D_rho + A_z(x)I(x)I  eq. (cylinder)

    disk_lambda: M = I (x) A_lambda + A_theta (x) D_rho^lambda     Section 5.3

    D_rho = diag(rho_i^-2), D_phi = diag(sin^-2 phi_k), D_rho^lambda =
    diag(rho_i^(-2-lambda)) (lambda = extent[1]).  A sphere of radius rho_*
    carries the factor rho_*^-2 on both terms.
    """
    ops = op.operators_1d(geometry, n, extent)
    A, g = ops["A"], ops["grid"]
    if geometry == "disk_lambda":
        Ar, At = A
        Dr = np.diag(g[0] ** (-2.0 - extent[1]))
        return [_kron(np.eye(n[1]), Ar), _kron(At, Dr)]
    if geometry == "disk":
        Ar, At = A
        Dr = np.diag(g[0] ** -2.0)
        I_t = np.eye(n[1])
        return [_kron(I_t, Ar), _kron(At, Dr)]
    if geometry == "sphere":
        At, Ap = A
        Dp = np.diag(np.sin(g[1]) ** -2.0)
        s = extent[0] ** -2.0
        return [s * _kron(Dp, At), s * _kron(Ap, np.eye(n[0]))]
    if geometry == "ball":
        Ar, At, Ap = A
        Dr = np.diag(g[0] ** -2.0)
        Dp = np.diag(np.sin(g[2]) ** -2.0)
        I_r, I_t = np.eye(n[0]), np.eye(n[1])
        return [_kron(np.eye(n[2]), I_t, Ar), _kron(Dp, At, Dr), _kron(Ap, I_t, Dr)]
    if geometry == "cylinder":
        Ar, At, Az = A
        Dr = np.diag(g[0] ** -2.0)
        I_r, I_t, I_z = np.eye(n[0]), np.eye(n[1]), np.eye(n[2])
        return [_kron(I_z, I_t, Ar), _kron(I_z, At, Dr), _kron(Az, I_t, I_r)]
    raise ValueError(geometry)


def laplacian(geometry: str, n, extent=(1.0, 1.0)):
    """Assembled M (sparse)."""
    T = terms(geometry, n, extent)
    M = T[0]
    for t in T[1:]:
        M = M + t
    return M.tocsr()


def dirichlet_lift(geometry: str, n, extent=(1.0, 1.0)) -> np.ndarray:
    """Vector r with M w + r * w_D the discrete Laplacian when w = w_D at z_*.

    The cylinder has a Dirichlet end at z_* (Table 1) and the anomalous disk
    one at rho_* (Section 5.3); elsewhere r = 0.
    """
    if geometry == "disk_lambda":
        nr, nt = n
        er = np.zeros(nr)
        er[-1] = op.rho_lambda_boundary(nr, extent[1], extent[0])
        return np.kron(np.ones(nt), er)
    if geometry != "cylinder":
        return np.zeros(int(np.prod(n)))
    nr, nt, nz = n
    ez = op.z_boundary_column(nz, extent[1])
    return np.kron(ez, np.ones(nr * nt))


def vec(W: np.ndarray) -> np.ndarray:
    """Paper vectorisation: first index fastest."""
    return np.asarray(W).ravel(order="F")


def unvec(w: np.ndarray, n) -> np.ndarray:
    return np.asarray(w).reshape(tuple(n), order="F")


def from_layout(field: np.ndarray) -> np.ndarray:
    """[.., n3, n2, n1] C-contiguous storage  ->  array indexed [i, j, k]."""
    nd = field.ndim
    return np.transpose(field, tuple(range(nd - 1, -1, -1)))


def to_layout(W: np.ndarray) -> np.ndarray:
    nd = W.ndim
    return np.ascontiguousarray(np.transpose(W, tuple(range(nd - 1, -1, -1))))
