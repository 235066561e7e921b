"""Split exponential Euler in matrix / tensor form (paper Section 4).

One step for species s of an N-coupled system (eq. (BVAM_SExpE)):

    F_s     = d_s M W_s + G_s(W_1, ..., W_N)
    W_s^+   = W_s + tau * phi_1(tau d_s M_1) ... phi_1(tau d_s M_d) F_s

where M = M_1 + ... + M_d is the Kronecker sum of ``assemble.terms``; the
rightmost factor (M_d) acts first (eq. (splitorder); the order matters).
Each factor is applied as a mu-mode product (``mode_product``) following
eqs. (ee_disk), (ee_sphere), (ee_ball) and (ee_cylinder):

* an unscaled mode (A_rho, A_phi on the sphere, A_z) by the dense matrix
  phi_1(tau d A) obtained by diagonalisation;
* a mode scaled by another coordinate (A_theta with D_rho / D_phi, A_phi
  with D_rho in the ball) through its eigenbasis: a mode product with the
  inverse eigenvector matrix, a Hadamard product with the tensor of scalar
  phi_1 values, and a mode product with the eigenvector matrix.

Eigenpairs come from numpy's LAPACK eigensolver applied to the symmetrised
operator (Proposition 1), including for A_theta (no closed form is used).
"""
from __future__ import annotations

import numpy as np

from . import assemble, operators as op, reactions
from .phi import eig_tridiag, phi1_dense_expm, phi1_matrix, phi1_scalar


def mode_product(X: np.ndarray, L: np.ndarray, mu: int) -> np.ndarray:
    """Y = X x_mu L :  Y[.., l, ..] = sum_k L[l, k] X[.., k, ..] (mu counted from 1)."""
    ax = mu - 1
    return np.moveaxis(np.tensordot(L, X, axes=(1, ax)), 0, ax)


class SplitEE:
    """Split exponential Euler for one geometry, grid and set of species.

    ``diff`` holds d_s per species.  ``extent`` = (rho_*, z_*); for the
    sphere rho_* is its radius (operator scaled by rho_*^-2); for
    "disk_lambda" the second entry is lambda (Section 5.3).
    """

    def __init__(self, geometry, n, diff, tau, extent=(1.0, 1.0)):
        self.geometry = geometry
        self.n = tuple(int(x) for x in n)
        self.diff = [float(d) for d in diff]
        self.tau = float(tau)
        self.extent = (float(extent[0]), float(extent[1]))
        ops = op.operators_1d(geometry, self.n, self.extent)
        self.A = ops["A"]
        self.grid = ops["grid"]
        self.M = assemble.laplacian(geometry, self.n, self.extent)
        self.lift = assemble.dirichlet_lift(geometry, self.n, self.extent)
        self._build_factors()

    # -- precompute (Section 4: "once and for all before the time marching") --
    def _build_factors(self):
        g, A, tau = self.geometry, self.A, self.tau
        self.f = []  # per species dict of factors
        if g in ("disk", "disk_lambda"):
            lam_t, Q, _ = eig_tridiag(A[1])
            # D_rho: rho^-2, or rho^(-2-lambda) for the anomalous operator
            rinv2 = self.grid[0] ** (-2.0 - (self.extent[1] if g == "disk_lambda" else 0.0))
            for d in self.diff:
                self.f.append({
                    "P_rho": phi1_matrix(A[0], tau * d),
                    "Phi_rt": phi1_scalar(tau * d * np.outer(rinv2, lam_t)),
                })
            self.Q = Q
        elif g == "sphere":
            lam_t, Q, _ = eig_tridiag(A[0])
            s2 = self.extent[0] ** -2.0
            sinv2 = np.sin(self.grid[1]) ** -2.0
            for d in self.diff:
                self.f.append({
                    "P_phi": phi1_matrix(A[1], tau * d * s2),
                    "Phi_tp": phi1_scalar(tau * d * s2 * np.outer(lam_t, sinv2)),
                })
            self.Q = Q
        elif g == "ball":
            lam_t, Q, _ = eig_tridiag(A[1])
            lam_p, Vp, Vpinv = eig_tridiag(A[2])
            rinv2 = self.grid[0] ** -2.0
            sinv2 = np.sin(self.grid[2]) ** -2.0
            for d in self.diff:
                self.f.append({
                    "P_rho": phi1_matrix(A[0], tau * d),
                    # Phi_{rho,.,phi}(i,k) = phi_1(tau d rho_i^-2 lambda_phi_k)
                    "Phi_rp": phi1_scalar(tau * d * np.outer(rinv2, lam_p)),
                    # Phi_{rho,theta,phi}(i,j,k) = phi_1(tau d rho_i^-2 lambda_theta_j sin^-2 phi_k)
                    "Phi_rtp": phi1_scalar(tau * d * rinv2[:, None, None]
                                           * lam_t[None, :, None] * sinv2[None, None, :]),
                })
            self.Q, self.Vp, self.Vpinv = Q, Vp, Vpinv
        elif g == "cylinder":
            lam_t, Q, _ = eig_tridiag(A[1])
            rinv2 = self.grid[0] ** -2.0
            for d in self.diff:
                self.f.append({
                    "P_rho": phi1_matrix(A[0], tau * d),
                    "P_z": phi1_matrix(A[2], tau * d),
                    "Phi_rt": phi1_scalar(tau * d * np.outer(rinv2, lam_t)),
                })
            self.Q = Q
        else:
            raise ValueError(g)

    # -- operator and split phi_1 action ------------------------------------
    def apply_M(self, W: np.ndarray, s: int = 0, w_dirichlet: float = 0.0) -> np.ndarray:
        """d_s (M W + lift * w_D) through the assembled sparse matrix."""
        w = assemble.vec(W)
        out = self.M @ w + self.lift * w_dirichlet
        return self.diff[s] * assemble.unvec(out, self.n)

    def split_phi1(self, F: np.ndarray, s: int = 0) -> np.ndarray:
        """phi_1(tau d_s M_1) ... phi_1(tau d_s M_d) F in the paper's tensor form."""
        g, f = self.geometry, self.f[s]
        if g in ("disk", "disk_lambda"):  # eq. (ee_disk): phi1(tau A_rho) (Phi o (F Q)) Q^T
            Y = f["Phi_rt"] * (F @ self.Q)
            return f["P_rho"] @ (Y @ self.Q.T)
        if g == "sphere":  # eq. (ee_sphere): Q (Phi o (Q^T F phi1(tau A_phi)^T))
            Y = f["Phi_tp"] * (self.Q.T @ F @ f["P_phi"].T)
            return self.Q @ Y
        if g == "ball":  # eq. (ee_ball)
            Y = mode_product(F, self.Vpinv, 3)
            Y = f["Phi_rp"][:, None, :] * Y
            Y = mode_product(Y, self.Vp, 3)
            Y = mode_product(Y, self.Q.T, 2)
            Y = f["Phi_rtp"] * Y
            Y = mode_product(Y, self.Q, 2)
            return mode_product(Y, f["P_rho"], 1)
        if g == "cylinder":  # eq. (ee_cylinder)
            Y = mode_product(F, f["P_z"], 3)
            Y = mode_product(Y, self.Q.T, 2)
            Y = f["Phi_rt"][:, :, None] * Y
            Y = mode_product(Y, self.Q, 2)
            return mode_product(Y, f["P_rho"], 1)
        raise ValueError(g)

    # -- one step of an N-coupled system ------------------------------------
    def step(self, Ws, reaction_fn, w_dirichlet=None, source=None):
        """W_s <- W_s + tau S_s (d_s M W_s + G_s) for every species s.

        ``reaction_fn(Ws) -> Gs``; ``source`` (optional list) is added to G;
        ``w_dirichlet`` gives the boundary value per species at z_* (cylinder).
        """
        G = reaction_fn(Ws)
        out = []
        for s, W in enumerate(Ws):
            wd = 0.0 if w_dirichlet is None else w_dirichlet[s]
            F = self.apply_M(W, s, wd) + G[s]
            if source is not None:
                F = F + source[s]
            out.append(W + self.tau * self.split_phi1(F, s))
        return out

    # -- dense references for tiny grids -------------------------------------
    def split_dense(self, s: int = 0) -> np.ndarray:
        """Prod_mu phi_1(tau d_s M_mu) assembled densely via block-matrix expm."""
        T = assemble.terms(self.geometry, self.n, self.extent)
        c = self.tau * self.diff[s]
        S = np.eye(self.M.shape[0])
        for Mmu in T:  # S = phi(M_1) phi(M_2) ... phi(M_d)
            S = S @ phi1_dense_expm(c * Mmu.toarray())
        return S


def make(workload, n=None, tau=None):
    """SplitEE for a ``workloads.Workload`` (optionally on another grid / tau)."""
    return SplitEE(workload.geometry, n or workload.n, workload.diff,
                   workload.tau if tau is None else tau, workload.extent)


def initial_state(workload, perturbation: np.ndarray):
    """Species arrays [i,j(,k)] = equilibrium + perturbation (storage layout in)."""
    eq = reactions.equilibrium(workload.reaction, workload.params)
    return [eq[s] + assemble.from_layout(perturbation[s]) for s in range(workload.n_species)]


def run(workload, perturbation: np.ndarray, steps: int, n=None, callback=None):
    """Integrate a workload from equilibrium + perturbation; returns species arrays."""
    se = make(workload, n)
    eq = reactions.equilibrium(workload.reaction, workload.params)
    Ws = initial_state(workload, perturbation)
    wd = eq if workload.geometry in ("cylinder", "disk_lambda") else None
    react = lambda U: reactions.reaction(workload.reaction, U, workload.params)  # noqa: E731
    for it in range(steps):
        Ws = se.step(Ws, react, w_dirichlet=wd)
        if callback is not None:
            callback(it + 1, Ws)
    return Ws


def stack_layout(Ws) -> np.ndarray:
    """Species list [i,j,k] -> storage layout [species][k][j][i]."""
    return np.stack([assemble.to_layout(W) for W in Ws])
