"""Pins of the bulk-surface ball + sphere system (paper Section 5.5) and of
the reading of its Robin coupling (ghost point in the ball's boundary row):

* the ghost-point boundary row is exact on rho^2 (Delta = 6, d/drho = 2 rho)
  and second-order on rho^4;
* with the kinetics off, the discrete total mass of each species pair,
  sum(omega_B u) + sum(omega_S r) with omega the left null vectors of the
  two Laplacians, is conserved step by step, and the surface weight this
  requires, kappa * omega_rho[n], tends to the sphere's area element
  (rho_*^2 per solid angle against rho^2 drho in the ball);
* the homogeneous equilibrium is a fixed point of the full system;
* the coupling terms agree with an independently assembled sparse operator
  of the linear coupled system.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.linalg import null_space

from oracle import assemble, bulk_surface as BS, operators as op


def _left_null(A):
    w = null_space(A.T)[:, 0]
    return w / w.sum()


def test_ghost_point_row_on_polynomials():
    for n in (8, 16, 31):
        r = op.rho_grid(n, 3)
        A = op.A_rho(n, 3)
        got = A @ r**2
        got[-1] += BS.kappa(n) * 2.0
        np.testing.assert_allclose(got, 6.0, rtol=1e-12)
    # on rho^4 the interior rows are second order; the boundary row, like the
    # paper's own ghost-point Neumann row, is first order (its ghost value
    # misses the h^3 f_rhorhorho / 3 term), which still gives a second-order
    # solution
    inner, edge = [], []
    for n in (20, 40, 80):
        r = op.rho_grid(n, 3)
        got = op.A_rho(n, 3) @ r**4
        got[-1] += BS.kappa(n) * 4.0
        err = np.abs(got - 20.0 * r**2)
        inner.append(err[:-1].max())
        edge.append(err[-1])
    assert 3.5 < inner[0] / inner[1] < 4.5 and 3.5 < inner[1] / inner[2] < 4.5, inner
    assert 1.8 < edge[0] / edge[1] < 2.2 and 1.8 < edge[1] / edge[2] < 2.2, edge


@pytest.mark.parametrize("n", [(6, 8, 7), (9, 12, 10)])
def test_mass_conservation_without_kinetics(n):
    sys = BS.BulkSurface(n, 2e-3, kinetics=False)
    w_rho = _left_null(op.A_rho(n[0], 3))
    w_phi = _left_null(op.A_phi(n[2]))
    w_theta = np.ones(n[1]) / n[1]
    wb = np.multiply.outer(np.multiply.outer(w_rho, w_theta), w_phi)
    ws = sys.kappa * w_rho[-1] * np.multiply.outer(w_theta, w_phi)
    rng = np.random.default_rng(4)
    U = [1.0 + 0.3 * rng.random(n), 0.8 + 0.3 * rng.random(n)]
    S = [1.1 + 0.3 * rng.random(n[1:]), 0.7 + 0.3 * rng.random(n[1:])]
    tot = [np.sum(wb * U[q]) + np.sum(ws * S[q]) for q in range(2)]
    moved = 0.0
    for _ in range(5):
        U1, S1 = sys.step(U, S)
        moved = max(moved, max(abs(np.sum(ws * (S1[q] - S[q]))) for q in range(2)))
        U, S = U1, S1
        for q in range(2):
            assert abs(np.sum(wb * U[q]) + np.sum(ws * S[q]) - tot[q]) < 1e-13 * abs(tot[q])
    assert moved > 1e-6  # mass did move between bulk and surface


def test_surface_weight_is_the_area_element():
    """kappa * omega_rho[n] / sum(omega_rho) = rho_*^2 / (rho_*^3 / 3) = 3:
    the weight conservation asks of the surface is the sphere's area element
    against the ball's discrete volume measure, exactly on every grid."""
    for nr in (3, 16, 33, 64):
        w = _left_null(op.A_rho(nr, 3))
        assert abs(BS.kappa(nr) * w[-1] - 3.0) < 1e-12


def test_equilibrium_is_a_fixed_point():
    sys = BS.BulkSurface((7, 10, 9), 1e-4)
    eb, es = BS.equilibrium()
    n = sys.n
    U = [np.full(n, eb[0]), np.full(n, eb[1])]
    S = [np.full(n[1:], es[0]), np.full(n[1:], es[1])]
    U1, S1 = sys.step(U, S)
    for a, b in zip(U1 + S1, U + S):
        assert np.abs(a - b).max() < 1e-13


def test_coupling_against_assembled_operator():
    """F of the linear coupled system (kinetics off) = K [u; v; r; s] with K
    assembled as one sparse matrix: diffusion blocks plus the Robin entries
    of the boundary layer and the exchange entries of the surface."""
    n = (5, 6, 7)
    p = BS.PARAMS
    sys = BS.BulkSurface(n, 1e-3, kinetics=False)
    Mb = assemble.laplacian("ball", n)
    Ms = assemble.laplacian("sphere", n[1:])
    Nb, Ns = Mb.shape[0], Ms.shape[0]
    # boundary-layer points of the ball in vec order (i fastest): i = n1 - 1
    bidx = np.arange(Ns) * n[0] + (n[0] - 1)
    E = sp.csr_matrix((np.ones(Ns), (bidx, np.arange(Ns))), shape=(Nb, Ns))  # surface -> layer
    k, z1 = sys.kappa, p["zeta1"]
    Kuu = Mb - k * z1 * p["zeta3"] * (E @ E.T)
    Kvv = p["delta"] * Mb - k * z1 * p["eta2"] * (E @ E.T)
    Kur = k * z1 * p["zeta2"] * E
    Kvs = k * z1 * p["eta1"] * E
    Krr = Ms - z1 * p["zeta2"] * sp.identity(Ns)
    Kss = p["epsilon"] * Ms - z1 * p["eta1"] * sp.identity(Ns)
    Kru = z1 * p["zeta3"] * E.T
    Ksv = z1 * p["eta2"] * E.T
    Z = lambda a, b: sp.csr_matrix((a, b))  # noqa: E731
    K = sp.bmat([[Kuu, Z(Nb, Nb), Kur, Z(Nb, Ns)],
                 [Z(Nb, Nb), Kvv, Z(Nb, Ns), Kvs],
                 [Kru, Z(Ns, Nb), Krr, Z(Ns, Ns)],
                 [Z(Ns, Nb), Ksv, Z(Ns, Ns), Kss]]).tocsr()
    rng = np.random.default_rng(8)
    U = [rng.random(n), rng.random(n)]
    S = [rng.random(n[1:]), rng.random(n[1:])]
    Gb, Gs = sys.reactions(U, S)
    F = [sys.ball.apply_M(U[q], q) + Gb[q] for q in range(2)] + \
        [sys.surface.apply_M(S[q], q) + Gs[q] for q in range(2)]
    x = np.concatenate([assemble.vec(a) for a in U + S])
    ref = K @ x
    got = np.concatenate([assemble.vec(a) for a in F])
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
