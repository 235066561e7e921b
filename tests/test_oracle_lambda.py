"""Pins of the anomalous-diffusion disk (paper Section 5.3, eqs. (anomalous),
(A_lambda), Appendix "On the discretization matrix of Delta_lambda").

* lambda = 0: the entries are those of the polar Laplacian on the Dirichlet
  half-point grid, written out here independently, and the spectrum of the
  assembled operator converges at second order to -j_{m,k}^2 (zeros of J_m);
* any lambda: second-order consistency with the continuous operator on a
  function vanishing at rho_*, zero row sums except the Dirichlet row, and
  the Appendix's closed-form symmetriser makes Xi^-1 A Xi symmetric;
* the split step: equality with the dense Kronecker product on tiny grids,
  the lifted equilibrium is a fixed point, and the gradient oracle agrees
  with central differences.
"""
import math

import numpy as np
import pytest
from scipy.special import jn_zeros

from oracle import adjoint, assemble, operators as op, reactions as R, splitee
import workloads

LAMS = [-1.95, -0.7, 0.0, 0.5]


def test_lambda_zero_entries():
    n = 9
    h = 1.0 / (n + 0.5)
    A = op.A_rho_lambda(n, 0.0)
    l = np.arange(1, n)
    np.testing.assert_allclose(np.diag(A), -2.0 / h**2, rtol=1e-14)
    np.testing.assert_allclose(np.diag(A, 1), 2 * l / ((2 * l - 1) * h**2), rtol=1e-14)
    np.testing.assert_allclose(np.diag(A, -1), 2 * l / ((2 * l + 1) * h**2), rtol=1e-14)
    np.testing.assert_allclose(op.rho_lambda_grid(n, 0.0), h / 2 + h * np.arange(n), rtol=1e-15)
    # the boundary rho_* = 1 is the next grid point after the last one
    assert abs(op.rho_lambda_grid(n, 0.0)[-1] + h - 1.0) < 1e-15


def test_lambda_zero_dirichlet_bessel_spectrum():
    """Eigenvalues of the assembled lambda = 0 operator -> -j_{m,k}^2, O(h^2)."""
    errs = []
    for nr in (16, 32):
        nt = 2 * nr
        M = assemble.laplacian("disk_lambda", (nr, nt), (1.0, 0.0)).toarray()
        ev = np.sort(-np.linalg.eigvals(M).real)[:6]
        # theta modes m >= 1 are double
        ref = np.sort(np.concatenate([jn_zeros(0, 3) ** 2] + [np.repeat(jn_zeros(m, 3) ** 2, 2)
                                                              for m in range(1, 4)]))[:6]
        errs.append(np.abs(ev - ref) / ref)
    ratio = errs[0].max() / errs[1].max()
    assert errs[1].max() < 5e-3 and 3.0 < ratio < 5.0, (errs, ratio)


@pytest.mark.parametrize("lam,low,high", [(-1.95, 3.5, 4.5), (-0.7, 3.5, 4.5), (0.0, 3.5, 4.5),
                                          (0.5, 2.5, 4.5)])
def test_consistency_order(lam, low, high):
    """A_lambda f vs Delta_lambda f = -p (p - lambda) rho^(p-2-lambda) for
    f = 1 - rho^p, which vanishes at rho_* = 1 (so the lift adds nothing):
    second order for lambda <= 0 (the paper's superdiffusive regime); for
    subdiffusion (lambda > 0) the rho^-lambda weight drops it to order 3/2
    at the first point."""
    p = 4.0
    errs = []
    for n in (40, 80):
        r = op.rho_lambda_grid(n, lam)
        A = op.A_rho_lambda(n, lam)
        exact = -p * (p - lam) * r ** (p - 2.0 - lam)
        errs.append(np.abs(A @ (1.0 - r**p) - exact).max() / np.abs(exact).max())
    assert low < errs[0] / errs[1] < high, errs


@pytest.mark.parametrize("lam", LAMS)
def test_row_sums_sign_pattern_and_spectrum(lam):
    n = 12
    A = op.A_rho_lambda(n, lam)
    rows = A.sum(axis=1)
    assert np.abs(rows[:-1]).max() < 1e-12 * np.abs(A).max()
    # the Dirichlet row: its sum is minus the coefficient of the boundary value
    assert abs(rows[-1] + op.rho_lambda_boundary(n, lam)) < 1e-12 * np.abs(A).max()
    assert (np.diag(A, 1) > 0).all() and (np.diag(A, -1) > 0).all()
    ev = np.linalg.eigvals(A)
    assert np.abs(ev.imag).max() < 1e-9 * np.abs(ev).max() and (ev.real < 0).all()


@pytest.mark.parametrize("lam", [-1.95, -0.7])
def test_appendix_symmetriser(lam):
    """xi_1 = 1, xi_l^2 = (1-lam)^(1+lam) / ((2l-1)-lam)^(1+lam) * (l-1)! / prod_{i<l} (i - lam):
    Xi^-1 A Xi is symmetric, and max Xi^-1 grows like sqrt(n)."""
    def xi(n):
        x = np.ones(n)
        for l in range(2, n + 1):
            # in logarithms: (l-1)! and the product overflow for large l
            lg = (1 + lam) * (math.log(1 - lam) - math.log((2 * l - 1) - lam))
            lg += sum(math.log(i) - math.log(i - lam) for i in range(1, l))
            x[l - 1] = math.exp(0.5 * lg)
        return x
    n = 20
    X = xi(n)
    S = (op.A_rho_lambda(n, lam) * X[None, :]) / X[:, None]
    assert np.abs(S - S.T).max() < 1e-12 * np.abs(S).max()
    big = [1.0 / xi(m).min() for m in (50, 200)]
    assert 1.7 < big[1] / big[0] < 2.3  # factor sqrt(4) = 2


@pytest.mark.parametrize("lam", [-1.95, 0.5])
@pytest.mark.parametrize("tau", [1e-3, 0.05])
def test_split_action_equals_dense_kronecker(lam, tau):
    n = (5, 6)
    se = splitee.SplitEE("disk_lambda", n, [1.0, 7.5], tau, (1.0, lam))
    F = np.random.default_rng(11).standard_normal(n)
    for s in range(2):
        ref = assemble.unvec(se.split_dense(s) @ assemble.vec(F), n)
        got = se.split_phi1(F, s)
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_lifted_equilibrium_is_a_fixed_point():
    w = workloads.scaled(workloads.WORKLOADS["disk_lambda_160x160"], (10, 12))
    eq = R.equilibrium(w.reaction, w.params)
    g = R.reaction(w.reaction, [np.array([e]) for e in eq], w.params)
    assert max(abs(x[0]) for x in g) < 1e-12
    se = splitee.make(w)
    W = [np.full(w.n, e) for e in eq]
    out = se.step(W, lambda U: R.reaction(w.reaction, U, w.params), w_dirichlet=eq)
    assert max(np.abs(a - b).max() for a, b in zip(out, W)) < 1e-12


def _richardson(f, h):
    c1 = (f(h) - f(-h)) / (2 * h)
    c2 = (f(h / 2) - f(-h / 2)) / h
    return (4 * c2 - c1) / 3


def test_gradient_vs_central_differences():
    """Gradient oracle on the anomalous disk with the scaled kinetics
    (lifted Dirichlet term; parameters alpha_2, beta_1, alpha_1)."""
    w = workloads.scaled(workloads.WORKLOADS["disk_lambda_160x160"], (6, 8), steps=4)
    eq = R.equilibrium(w.reaction, w.params)
    pert = 1e-3 * np.random.default_rng(3).random(w.field_shape())
    W0 = [eq[s] + assemble.from_layout(pert[s]) for s in range(2)]
    target = W0[0] + 1e-3 * np.random.default_rng(4).random(w.n)
    L, lam0, gd, gp = adjoint.loss_and_grad(w, W0, target, w.steps, w_dirichlet=eq)
    h = 1e-4
    e = [np.random.default_rng(5 + s).standard_normal(w.n) for s in range(2)]
    an = sum(np.sum(lam0[s] * e[s]) for s in range(2))
    fd = _richardson(lambda t: adjoint.loss(w, [W0[s] + t * e[s] for s in range(2)], target, w.steps,
                                            w_dirichlet=eq), h)
    assert abs(fd - an) < 1e-8 * abs(an)
    scale = max(np.abs(gd).max(), np.abs(gp).max())
    for s in range(2):
        def f_d(t, s=s):
            d = list(w.diff)
            d[s] += t
            return adjoint.loss(w, W0, target, w.steps, diff=d, w_dirichlet=eq)
        assert abs(_richardson(f_d, h) - gd[s]) < 1e-6 * abs(gd[s]) + 1e-7 * scale
    for q in range(3):
        def f_p(t, q=q):
            p = list(w.params)
            p[q] += t * max(1.0, abs(p[q])) * 1e-2
            return adjoint.loss(w, W0, target, w.steps, params=p, w_dirichlet=eq)
        hq = max(1.0, abs(w.params[q])) * 1e-2
        assert abs(_richardson(f_p, h) / hq - gp[q]) < 1e-6 * abs(gp[q]) + 1e-7 * scale
