"""Pins of the oracle's split exponential Euler step (paper Section 4, 5.1).

* tiny grids: the mu-mode / Hadamard realisation equals the dense product
  phi_1(tau M_1) ... phi_1(tau M_d) built from scipy's expm of each
  assembled Kronecker term (an independent route), in the paper's order;
* exactness of the linear step for data on which a single term acts;
* steady states are fixed points; the split error is O(tau^2);
* whole scheme: the printed SplitEE errors of Figure 1.
"""
import math
import os

import numpy as np
import pytest
from scipy.special import iv

from oracle import assemble, operators as op, reactions as R, splitee
from oracle.phi import phi1_dense_expm

import workloads

TINY = [("disk", (5, 6)), ("sphere", (6, 5)), ("ball", (4, 5, 6)), ("cylinder", (4, 5, 3))]


@pytest.mark.parametrize("geometry,n", TINY)
@pytest.mark.parametrize("tau", [1e-3, 0.05])
def test_split_action_equals_dense_kronecker(geometry, n, tau):
    se = splitee.SplitEE(geometry, n, [1.0, 7.5], tau, (1.0, 1.4))
    rng = np.random.default_rng(11)
    F = rng.standard_normal(n)
    for s in range(2):
        S = se.split_dense(s)
        ref = assemble.unvec(S @ assemble.vec(F), n)
        got = se.split_phi1(F, s)
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("geometry,n", TINY)
def test_split_order_is_detectable(geometry, n):
    """Reversing the factor order changes the result (so the test above pins it)."""
    se = splitee.SplitEE(geometry, n, [3.0], 0.05)
    T = assemble.terms(geometry, n)
    rev = np.eye(se.M.shape[0])
    for Mmu in reversed(T):
        rev = rev @ phi1_dense_expm(se.tau * 3.0 * Mmu.toarray())
    F = np.random.default_rng(3).standard_normal(n)
    diff = np.abs(assemble.unvec(rev @ assemble.vec(F), n) - se.split_phi1(F, 0)).max()
    assert diff > 1e-6


@pytest.mark.parametrize("geometry,n", TINY)
def test_operator_tensor_vs_sparse(geometry, n):
    """d M W from the assembled matrix equals the sum of 1D stencils per mode."""
    se = splitee.SplitEE(geometry, n, [2.0], 0.01)
    W = np.random.default_rng(5).standard_normal(n)
    Ms = [se.A[m] for m in range(len(n))]
    g = se.grid
    mp = splitee.mode_product
    if geometry == "disk":
        ref = Ms[0] @ W + (g[0] ** -2.0)[:, None] * (W @ Ms[1].T)
    elif geometry == "sphere":
        ref = (Ms[0] @ W) * (np.sin(g[1]) ** -2.0)[None, :] + W @ Ms[1].T
    elif geometry == "ball":
        dr = (g[0] ** -2.0)[:, None, None]
        dp = (np.sin(g[2]) ** -2.0)[None, None, :]
        ref = mp(W, Ms[0], 1) + dr * dp * mp(W, Ms[1], 2) + dr * mp(W, Ms[2], 3)
    else:
        dr = (g[0] ** -2.0)[:, None, None]
        ref = mp(W, Ms[0], 1) + dr * mp(W, Ms[1], 2) + mp(W, Ms[2], 3)
    np.testing.assert_allclose(se.apply_M(W, 0), 2.0 * ref, atol=1e-10 * np.abs(ref).max())


@pytest.mark.parametrize("geometry,n,active", [
    ("disk", (9, 8), 0), ("sphere", (8, 9), 1), ("ball", (6, 4, 5), 0), ("cylinder", (6, 4, 7), 2)])
def test_linear_step_exact_single_active_mode(geometry, n, active):
    """With G = 0 and data varying only along one unscaled/radial coordinate,
    only that term of M acts and one step equals e^{tau d A} exactly."""
    d, tau = 1.7, 0.03
    se = splitee.SplitEE(geometry, n, [d], tau)
    f = np.cos(1.3 * np.arange(n[active]))
    shape = [1] * len(n)
    shape[active] = n[active]
    W = np.broadcast_to(f.reshape(shape), n).copy()
    Wn = se.step([W], lambda U: [np.zeros_like(U[0])])[0]
    from scipy.linalg import expm
    ef = expm(tau * d * se.A[active]) @ f
    ref = np.broadcast_to(ef.reshape(shape), n)
    assert np.abs(Wn - ref).max() < 1e-13


@pytest.mark.parametrize("geometry,n", TINY)
def test_constants_stationary(geometry, n):
    se = splitee.SplitEE(geometry, n, [1.0, 20.0], 0.1)
    W = [np.full(n, 0.7), np.full(n, -1.1)]
    out = se.step(W, lambda U: [np.zeros_like(U[0])] * 2, w_dirichlet=[0.7, -1.1])
    for a, b in zip(out, W):
        assert np.abs(a - b).max() < 1e-13


@pytest.mark.parametrize("kind,params", [("schnakenberg", (0.1, 0.9)),
                                         ("schnakenberg", (0.17, 0.8)),
                                         ("ais3", (0.1, 0.9, 0.5, 1.0))])
def test_equilibrium_is_fixed_point(kind, params):
    eq = R.equilibrium(kind, params)
    g = R.reaction(kind, [np.array([e]) for e in eq], params)
    assert max(abs(x[0]) for x in g) < 1e-15
    # and the equilibrium of the workload model is a fixed point of the step
    n = (4, 5, 3)
    se = splitee.SplitEE("cylinder", n, [1.0] * len(eq), 0.1)
    W = [np.full(n, e) for e in eq]
    out = se.step(W, lambda U: R.reaction(kind, U, params), w_dirichlet=eq)
    assert max(np.abs(a - b).max() for a, b in zip(out, W)) < 1e-13


def test_split_error_second_order_in_tau():
    """||phi_1(tau M) - phi_1(tau M_1) phi_1(tau M_2)|| = O(tau^2), eq. (splitorder)."""
    n = (5, 6)
    T = [t.toarray() for t in assemble.terms("disk", n)]
    M = T[0] + T[1]
    errs = []
    for tau in (2e-4, 1e-4):
        E = phi1_dense_expm(tau * M) - phi1_dense_expm(tau * T[0]) @ phi1_dense_expm(tau * T[1])
        errs.append(np.abs(E).max())
    assert 3.8 < errs[0] / errs[1] < 4.2


def _fig1_golden():
    path = os.path.join(os.path.dirname(__file__), "golden", "fig1_splitee_errors.txt")
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    return [((int(a), int(b)), int(m), float(e)) for a, b, m, e in rows]


def _fig1_error(n, m):
    """Relative error at t_* = 1 as read from Section 5.1.

    Reading: per component, the rho-weighted midpoint-rule L2 norm of the
    error on the grid divided by the exact L2 norm of the exact solution
    (||u(1)||^2 = e^-2 / 30 * 2 pi I_0(1/5), likewise v); the two relative
    errors are combined in the 2-norm.
    """
    p = R.BVAM_FIG1
    se = splitee.SplitEE("disk", n, [p["gamma"], p["delta"]], 1.0 / m)
    rho, th = se.grid
    RHO, TH = np.meshgrid(rho, th, indexing="ij")
    W = R.bvam_exact(0.0, RHO, TH)
    react = lambda U: R.bvam(U, p["alpha1"], p["alpha2"], p["alpha3"], p["beta1"], p["beta2"])  # noqa
    for it in range(m):
        W = se.step(W, react, source=R.bvam_sources(it * se.tau, RHO, TH))
    E = R.bvam_exact(1.0, RHO, TH)
    area = (rho[1] - rho[0]) * (th[1] - th[0])
    den = math.exp(-2.0) / 30.0 * 2.0 * math.pi * iv(0, 0.2)
    e = [math.sqrt(np.sum(RHO * (W[s] - E[s]) ** 2) * area / den) for s in range(2)]
    return math.hypot(*e)


@pytest.mark.parametrize("n,m,err", _fig1_golden())
def test_figure1_splitee_errors(n, m, err):
    got = _fig1_error(n, m)
    assert abs(got / err - 1.0) < 5e-4, (got, err)


def test_workload_initial_state_layout():
    w = workloads.scaled(workloads.WORKLOADS["ball_64x64x128"], (4, 5, 6))
    pert = workloads.perturbation(w)
    W = splitee.initial_state(w, pert)
    eq = R.equilibrium(w.reaction, w.params)
    assert W[0].shape == (4, 5, 6)
    assert W[1][3, 2, 1] == eq[1] + pert[1, 1, 2, 3]
    np.testing.assert_allclose(splitee.stack_layout(W) - np.array(eq)[:, None, None, None], pert,
                               rtol=0, atol=4e-16)
