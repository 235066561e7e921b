"""Each mu-mode product of the chain, alone on the GPU, against the same
product evaluated in float64 NumPy from the library's own host factors.

This isolates the kernel arithmetic (tiling, MFMA lane layouts, ragged
edges, epilogues) from the choice of factor route, which the parity tests
against the oracle cover."""
import numpy as np
import pytest

import paper_2604_11558_amd as tg
from oracle.splitee import mode_product as mp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _phi1(x):
    out = np.ones_like(x)
    nz = x != 0
    out[nz] = np.expm1(x[nz]) / x[nz]
    return out


def _chain_reference(geometry, n, grid, diff, tau):
    """List of callables (one per chain op) acting on [i,j,k] arrays, species s."""
    c = [grid.coords(m) for m in range(1, len(n) + 1)]
    if geometry == "disk":
        lt, Q, Qi = grid.eig(2)
        r2 = c[0] ** -2.0
        return [lambda X, d: _phi1(tau * d * np.outer(r2, lt)) * mp(X, Qi, 2),
                lambda X, d: mp(X, Q, 2),
                lambda X, d: mp(X, grid.phi1(1, tau * d), 1)]
    if geometry == "sphere":
        lt, Q, Qi = grid.eig(1)
        s2 = np.sin(c[1]) ** -2.0
        return [lambda X, d: mp(X, grid.phi1(2, tau * d), 2),
                lambda X, d: _phi1(tau * d * np.outer(lt, s2)) * mp(X, Qi, 1),
                lambda X, d: mp(X, Q, 1)]
    if geometry == "ball":
        lt, Q, Qi = grid.eig(2)
        lp, V, Vi = grid.eig(3)
        r2, s2 = c[0] ** -2.0, np.sin(c[2]) ** -2.0
        return [lambda X, d: _phi1(tau * d * np.outer(r2, lp))[:, None, :] * mp(X, Vi, 3),
                lambda X, d: mp(X, V, 3),
                lambda X, d: _phi1(tau * d * r2[:, None, None] * lt[None, :, None]
                                   * s2[None, None, :]) * mp(X, Qi, 2),
                lambda X, d: mp(X, Q, 2),
                lambda X, d: mp(X, grid.phi1(1, tau * d), 1)]
    lt, Q, Qi = grid.eig(2)
    r2 = c[0] ** -2.0
    return [lambda X, d: mp(X, grid.phi1(3, tau * d), 3),
            lambda X, d: _phi1(tau * d * np.outer(r2, lt))[:, :, None] * mp(X, Qi, 2),
            lambda X, d: mp(X, Q, 2),
            lambda X, d: mp(X, grid.phi1(1, tau * d), 1)]


@pytest.mark.parametrize("geometry,n", [("disk", (37, 70)), ("sphere", (70, 45)),
                                        ("ball", (20, 24, 37)), ("cylinder", (27, 30, 19)),
                                        ("ball", (64, 64, 128))])
@pytest.mark.parametrize("precision,tol", [("fp64", 2e-14), ("fp32", 3e-6)])
@pytest.mark.parametrize("tau", [5e-3, 0.3])
def test_chain_op_kernels(geometry, n, precision, tol, tau):
    diff = (1.0, 20.0)
    grid = tg.Grid(geometry, n)
    plan = tg.Plan(grid, diff, "schnakenberg", (0.1, 0.9), tau, precision)
    plan.set_route("generic")
    shape = plan.state_shape
    X = np.random.default_rng(8).random(shape)
    x = plan.state_from_deviation(X)
    y = torch.empty_like(x)
    refs = _chain_reference(geometry, n, grid, diff, tau)
    assert len(refs) == len(plan.chain_modes())
    worst = []
    for op, f in enumerate(refs):
        plan.apply_chain_op(op, x, y)
        got = y.double().cpu().numpy()[0]
        Xin = x.double().cpu().numpy()[0]  # the rounded input the kernel saw
        for s in range(2):
            Xs = np.transpose(Xin[s], tuple(range(len(n) - 1, -1, -1)))
            ref = f(Xs, diff[s])
            ref = np.transpose(ref, tuple(range(len(n) - 1, -1, -1)))
            err = float(np.abs(got[s] - ref).max() / np.abs(ref).max())
            worst.append((op, s, err))
    print(geometry, n, precision, tau, ["%d/%d:%.2e" % w for w in worst])
    assert max(w[2] for w in worst) < tol, worst
