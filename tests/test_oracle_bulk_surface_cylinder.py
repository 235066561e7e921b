"""Pins of the bulk-surface DIB system on the cylinder (paper Section 5.6)
and of the reading of its flux coupling (ghost point in A_z's z = 0 row):

* the DIB kinetics: eta4 of Sections 5.4 / 5.6 makes (r, s) = (0, zeta5) an
  equilibrium, the surface-only kinetics are eq. (DIBnl) (Section 5.4, the
  bulk values set to 1), and the Jacobians match central differences;
* the ghost-point row is exact on quadratics in z with the prescribed slope
  at z = 0, and first order on z^4 (second order inside), like the paper's
  own Neumann row;
* an exact discrete balance: with the trapezoid weights in z and the left
  null vector of the disk operator, sum w_B F_u + alpha3 sum w_D F_r equals
  the flux through the Dirichlet top plus the bulk kinetics (and likewise
  delta beta3 for v, s) -- the exchange creates no mass;
* the homogeneous equilibrium (alpha2, beta2, 0, zeta5) is a fixed point of
  the coupled step;
* the bulk F equals the plain cylinder F plus the flux computed from an
  explicit ghost layer (an independent assembly of the boundary row).
"""
import numpy as np
import pytest
from scipy.linalg import null_space

from oracle import bulk_surface as BS, operators as op, reactions as R

P = BS.DIB_CYL


def test_dib_equilibrium_and_section_5_4_kinetics():
    prm = BS.dib_params()
    pr, qs = R.dib_pq(P["alpha2"], P["beta2"], 0.0, P["zeta5"], *prm)
    assert abs(pr) < 1e-15 and abs(qs) < 1e-15
    # Section 5.4: eta4 = eta1 (1 - zeta5)(1 - eta3 + eta3 zeta5) / (zeta5 (1 + eta3 zeta5))
    e4 = R.dib_eta4(0.5, 5.0, 0.2)
    assert abs(e4 - 5.0 * 0.5 * 0.9 / (0.5 * 1.1)) < 1e-14
    sph = (10.0, 10.0, 1.0, 44.0, 0.5, 5.0, 2.5, 0.2, e4, 1.5)
    g = R.reaction("dib", [np.array(0.0), np.array(0.5)], sph)
    assert abs(g[0]) < 1e-14 and abs(g[1]) < 1e-13
    # surface-only kinetics = eq. (DIBnl) written out
    rng = np.random.default_rng(1)
    r, s = rng.random(20) - 0.5, rng.random(20)
    z1, z2, z3, z4, z5, e1, e2, e3, e4_, e5 = sph
    p_ref = z2 * (1 - s) * r - z3 * r**3 - z4 * (s - z5)
    q_ref = e1 * (1 + e2 * r) * (1 - s) * (1 - e3 * (1 - s)) - e4_ * s * (1 + e3 * s) * (1 + e5 * r)
    g = R.reaction("dib", [r, s], sph)
    np.testing.assert_allclose(g[0], z1 * p_ref, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(g[1], z1 * q_ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("kind,params,U", [
    ("dib", BS.dib_params(), [np.array([0.1, -0.3]), np.array([0.4, 0.7])]),
    ("linear", BS.linear_params(), [np.array([0.9, 1.3]), np.array([1.2, 0.2])])])
def test_kinetics_jacobians(kind, params, U):
    J = R.jacobian(kind, U, params)
    h = 1e-6
    for s in range(2):
        Up = [u.copy() for u in U]
        Um = [u.copy() for u in U]
        Up[s] += h
        Um[s] -= h
        gp, gm = R.reaction(kind, Up, params), R.reaction(kind, Um, params)
        for r in range(2):
            np.testing.assert_allclose(J[r][s], (gp[r] - gm[r]) / (2 * h), rtol=1e-7, atol=1e-8)


def test_ghost_row_on_polynomials_in_z():
    """(A_z u)_1 - (2/h) u'(0) is exact on quadratics and first order on
    z^3 + z^4 (the ghost value misses h^3 u_zzz(0) / 3); the interior rows
    are second order."""
    for n in (6, 13, 25):
        z = op.z_grid(n, 25.0)
        h = 25.0 / n
        g, c = 0.37, -0.011
        u = 1.0 + g * z + c * z * z
        got = op.A_z(n, 25.0) @ u
        got[0] += -(2.0 / h) * g
        got[-1] += (1.0 + g * 25.0 + c * 625.0) / h**2  # lifted Dirichlet value at z_*
        np.testing.assert_allclose(got, 2.0 * c, rtol=0, atol=1e-13 / h**2)
    edge, inner = [], []
    for n in (20, 40, 80):
        z = op.z_grid(n, 1.0)
        h = 1.0 / n
        got = op.A_z(n, 1.0) @ (z**3 + z**4)
        got[-1] += 2.0 / h**2  # lifted Dirichlet value u(1) = 2
        err = np.abs(got - (6.0 * z + 12.0 * z**2))
        edge.append(err[0])
        inner.append(err[1:].max())
    assert 1.8 < edge[0] / edge[1] < 2.2 and 1.8 < edge[1] / edge[2] < 2.2, edge
    assert 3.5 < inner[0] / inner[1] < 4.5 and 3.5 < inner[1] / inner[2] < 4.5, inner


def _weights(n, extent):
    A_disk = BS.SplitEE("disk", (n[0], n[1]), [1.0], 1.0, (extent[0], 1.0)).M.toarray()
    w = null_space(A_disk.T)[:, 0]
    w = w / w.sum()
    wD = w.reshape(n[1], n[0]).T  # vec order: rho fastest -> [i, j]
    hz = extent[1] / n[2]
    wz = np.full(n[2], hz)
    wz[0] = hz / 2.0
    return wD, np.multiply.outer(wD, wz), hz


@pytest.mark.parametrize("n,extent", [((6, 8, 5), (15.0, 25.0)), ((9, 7, 11), (1.3, 2.0))])
@pytest.mark.parametrize("kinetics", [False, True])
def test_discrete_balance_of_the_exchange(n, extent, kinetics):
    sys = BS.BulkSurfaceCylinder(n, 1e-2, extent, kinetics=kinetics)
    wD, wB, hz = _weights(n, extent)
    rng = np.random.default_rng(7)
    U = [1.0 + 0.2 * rng.random(n), 0.9 + 0.2 * rng.random(n)]
    S = [0.1 * rng.random(n[:2]), 0.5 + 0.1 * rng.random(n[:2])]
    Fb, Fs = sys.F(U, S)
    top = [(P["alpha2"] - U[0][:, :, -1]) / hz, (P["beta2"] - U[1][:, :, -1]) / hz]
    kin = R.linear(U, *BS.linear_params()) if kinetics else [0.0 * U[0], 0.0 * U[1]]
    for s, (d, c) in enumerate(((1.0, P["alpha3"]), (P["delta"], P["beta3"]))):
        lhs = float(np.sum(wB * Fb[s]) + d * c * np.sum(wD * Fs[s]))
        rhs = float(d * np.sum(wD * top[s]) + np.sum(wB * kin[s]))
        scale = float(np.sum(wB * np.abs(Fb[s])) + np.sum(wD * np.abs(Fs[s])))
        assert abs(lhs - rhs) < 1e-13 * scale, (s, lhs, rhs, scale)


def test_equilibrium_is_a_fixed_point():
    n = (7, 9, 6)
    sys = BS.BulkSurfaceCylinder(n, 0.025)
    ub, us = BS.cylinder_equilibrium()
    U = [np.full(n, ub[0]), np.full(n, ub[1])]
    S = [np.full(n[:2], us[0]), np.full(n[:2], us[1])]
    for _ in range(3):
        U, S = sys.step(U, S)
    for a, v in zip(U + S, ub + us):
        np.testing.assert_allclose(a, v, rtol=0, atol=1e-13)


def test_flux_row_against_an_explicit_ghost_layer():
    """Bulk F on z = 0 from a ghost layer u_0 = u_2 - 2 h_z du/dz(0) and the
    plain interior three-point z stencil (plus the (rho, theta) part)."""
    n, extent = (6, 8, 7), (15.0, 25.0)
    sys = BS.BulkSurfaceCylinder(n, 1e-2, extent, kinetics=False)
    rng = np.random.default_rng(9)
    U = [1.0 + 0.2 * rng.random(n), 0.9 + 0.2 * rng.random(n)]
    S = [0.1 * rng.random(n[:2]), 0.5 + 0.1 * rng.random(n[:2])]
    Fb, _ = sys.F(U, S)
    pr, qs = sys.pq(U, S)
    hz = extent[1] / n[2]
    disk = BS.SplitEE("disk", (n[0], n[1]), [1.0], 1.0, (extent[0], 1.0))
    for s, (d, slope) in enumerate(((1.0, P["zeta1"] * P["alpha3"] * pr),
                                    (P["delta"], P["zeta1"] * P["beta3"] * qs))):
        u0, u1, u2 = U[s][:, :, 0], U[s][:, :, 0], U[s][:, :, 1]
        ghost = u2 - 2.0 * hz * slope
        zpart = (ghost - 2.0 * u1 + u2) / hz**2
        rt = disk.apply_M(u0, 0)
        np.testing.assert_allclose(Fb[s][:, :, 0], d * (zpart + rt), rtol=1e-12,
                                   atol=1e-12 * np.abs(d * zpart).max())


def test_deviation_form_steps_the_same_map():
    n = (8, 10, 7)
    sys = BS.BulkSurfaceCylinder(n, 0.025)
    ub, us = BS.cylinder_equilibrium()
    rng = np.random.default_rng(11)
    dU = [1e-2 * rng.random(n) for _ in range(2)]
    dS = [1e-2 * rng.random(n[:2]) for _ in range(2)]
    U = [ub[s] + dU[s] for s in range(2)]
    S = [us[s] + dS[s] for s in range(2)]
    for _ in range(5):
        U, S = sys.step(U, S)
        dU, dS = sys.step_deviation(dU, dS)
    for a, d, v in zip(U + S, dU + dS, ub + us):
        np.testing.assert_allclose(a, v + d, rtol=0, atol=1e-12)
