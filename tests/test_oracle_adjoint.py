"""Pins of the gradient oracle (discrete adjoint of the split step).

* the op chain reproduces the tensor-form split action;
* dot-product identity <S x, y> = <x, S^T y>;
* the d-derivative of the chain and the full gradient against central
  finite differences in float64.
"""
import numpy as np
import pytest

from oracle import adjoint, splitee
import workloads

GEOMS = [("disk", (5, 7)), ("sphere", (6, 5)), ("ball", (4, 5, 6)), ("cylinder", (4, 5, 3))]


@pytest.mark.parametrize("geometry,n", GEOMS)
def test_chain_matches_split_and_transpose(geometry, n):
    se = splitee.SplitEE(geometry, n, [1.3, 9.0], 0.02)
    rng = np.random.default_rng(1)
    x, y = rng.standard_normal(n), rng.standard_normal(n)
    for s in range(2):
        ops = adjoint.chain(se, s)
        Sx = adjoint.apply_chain(ops, x)
        np.testing.assert_allclose(Sx, se.split_phi1(x, s), atol=1e-13)
        lhs = np.sum(Sx * y)
        rhs = np.sum(x * adjoint.apply_chain_T(ops, y))
        assert abs(lhs - rhs) < 1e-13 * max(1.0, abs(lhs))


@pytest.mark.parametrize("geometry,n", GEOMS)
def test_chain_derivative_in_d(geometry, n):
    d, h = 4.0, 1e-4
    x = np.random.default_rng(2).standard_normal(n)
    dd = adjoint.apply_chain_dd(adjoint.chain(splitee.SplitEE(geometry, n, [d], 0.02), 0), x)
    p = splitee.SplitEE(geometry, n, [d + h], 0.02).split_phi1(x, 0)
    m = splitee.SplitEE(geometry, n, [d - h], 0.02).split_phi1(x, 0)
    np.testing.assert_allclose(dd, (p - m) / (2 * h), atol=1e-8 * np.abs(dd).max())


def _richardson(f, h):
    """Central difference with one Richardson step (error O(h^4))."""
    c1 = (f(h) - f(-h)) / (2 * h)
    c2 = (f(h / 2) - f(-h / 2)) / h
    return (4 * c2 - c1) / 3, c1


def test_gradient_vs_central_differences():
    w = workloads.scaled(workloads.WORKLOADS["disk_256x512"], (6, 8), steps=5)
    pert = workloads.perturbation(w)
    W0 = splitee.initial_state(w, pert)
    target = W0[0] + 1e-3 * np.random.default_rng(7).random(w.n)
    L, lam0, gd, gp = adjoint.loss_and_grad(w, W0, target, w.steps)
    h = 1e-4
    dirs = [np.random.default_rng(9).standard_normal(w.n) for _ in range(2)]
    ic = lambda e: adjoint.loss(w, [W0[0] + e * dirs[0], W0[1] + e * dirs[1]], target, w.steps)  # noqa
    an = np.sum(lam0[0] * dirs[0]) + np.sum(lam0[1] * dirs[1])
    rich, plain = _richardson(ic, h)
    assert abs(plain - an) < 1e-5 * abs(an)  # plain central difference, h = 1e-4
    assert abs(rich - an) < 1e-9 * abs(an)
    scale = max(np.abs(gd).max(), np.abs(gp).max())
    for s in range(2):
        def fd(e, s=s):
            d = list(w.diff)
            d[s] += e
            return adjoint.loss(w, W0, target, w.steps, diff=d)
        rich, _ = _richardson(fd, h)
        assert abs(rich - gd[s]) < 1e-6 * abs(gd[s]) + 1e-7 * scale
    for q in range(2):
        def fp(e, q=q):
            p = list(w.params)
            p[q] += e
            return adjoint.loss(w, W0, target, w.steps, params=p)
        rich, _ = _richardson(fp, h)
        assert abs(rich - gp[q]) < 1e-6 * abs(gp[q]) + 1e-7 * scale


def test_gradient_cylinder_dirichlet_ais3_vs_central_differences():
    """Three species (AIS3) on the cylinder with the lifted Dirichlet data at z_*:
    the lift term enters F and dL/dd_s; kappa and mu enter through dG/dp."""
    w = workloads.scaled(workloads.WORKLOADS["cylinder_100x100x100"], (4, 5, 3), steps=4)
    pert = workloads.perturbation(w)
    W0 = splitee.initial_state(w, pert)
    # boundary data away from equilibrium, so the lift term does not vanish
    wd = [W0[s].mean() + 0.05 * (s + 1) for s in range(3)]
    target = W0[0] + 1e-3 * np.random.default_rng(11).random(w.n)
    L, lam0, gd, gp = adjoint.loss_and_grad(w, W0, target, w.steps, w_dirichlet=wd)
    h = 1e-4
    dirs = [np.random.default_rng(12 + s).standard_normal(w.n) for s in range(3)]
    ic = lambda e: adjoint.loss(w, [W0[s] + e * dirs[s] for s in range(3)], target, w.steps,  # noqa
                                w_dirichlet=wd)
    an = sum(np.sum(lam0[s] * dirs[s]) for s in range(3))
    rich, _ = _richardson(ic, h)
    assert abs(rich - an) < 1e-8 * abs(an)
    scale = max(np.abs(gd).max(), np.abs(gp).max())
    for s in range(3):
        def fd(e, s=s):
            d = list(w.diff)
            d[s] += e
            return adjoint.loss(w, W0, target, w.steps, diff=d, w_dirichlet=wd)
        rich, _ = _richardson(fd, h)
        assert abs(rich - gd[s]) < 1e-6 * abs(gd[s]) + 1e-7 * scale
    for q in range(4):
        def fp(e, q=q):
            p = list(w.params)
            p[q] += e
            return adjoint.loss(w, W0, target, w.steps, params=p, w_dirichlet=wd)
        rich, _ = _richardson(fp, h)
        assert abs(rich - gp[q]) < 1e-6 * abs(gp[q]) + 1e-7 * scale


def test_rounding_model_of_the_reverse_sweep():
    """round_to=float64 changes nothing; round_to=float32 moves lambda and
    the gradients by amounts of FP32 size (more than FP64 rounding, far less
    than the values), so the model neither vanishes nor swamps the result."""
    from types import SimpleNamespace
    from oracle import assemble, reactions
    n = (9, 12)
    wl = SimpleNamespace(geometry="disk", reaction="schnakenberg", tau=0.02, extent=(1.0, 1.0),
                         diff=(1.0, 20.0), params=(0.1, 0.9), n=n)
    eq = reactions.equilibrium("schnakenberg", (0.1, 0.9))
    rng = np.random.default_rng(3)
    W0 = [eq[s] + 1e-3 * rng.random(n) for s in range(2)]
    target = W0[0] + 1e-3 * rng.random(n)
    ref = adjoint.loss_and_grad(wl, W0, target, 3)
    same = adjoint.loss_and_grad(wl, W0, target, 3, round_to=np.float64)
    low = adjoint.loss_and_grad(wl, W0, target, 3, round_to=np.float32)
    for a, b in zip(ref[1], same[1]):
        np.testing.assert_array_equal(a, b)
    lam_r, lam_l = np.stack(ref[1]), np.stack(low[1])
    e = np.abs(lam_l - lam_r).max() / np.abs(lam_r).max()
    assert 1e-10 < e < 1e-4, e
    g_r = np.concatenate([ref[2], ref[3]])
    g_l = np.concatenate([low[2], low[3]])
    assert np.abs(g_l - g_r).max() < 1e-4 * np.abs(g_r).max()
