"""Bulk-surface ball + sphere system (Section 5.5) on the device, through the
C interface, against the FP64 oracle: every route of the bulk plan, FP64 and
FP32, the paper's 30 x 50 x 30 grid, graph-replayed runs against single
steps, and exact discrete mass conservation when only the exchange acts."""
import numpy as np
import pytest
from scipy.linalg import null_space

import paper_2604_11558_amd as tg
import workloads
from gpu_helpers import rel_err
from oracle import assemble, bulk_surface as BS, operators as op

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

P = BS.PARAMS
COUPLING = (P["zeta1"], P["zeta2"], P["zeta3"], P["eta1"], P["eta2"])


class Pair:
    def __init__(self, n, precision, tau=1e-4, seed=9, amplitude=1e-3, kinetics=True):
        self.n, self.tau = tuple(n), tau
        react = "schnakenberg_scaled" if kinetics else "none"
        pb = (P["alpha2"], P["beta1"], P["alpha1"]) if kinetics else ()
        ps = (P["alpha2"], P["beta1"], P["zeta1"]) if kinetics else ()
        self.bulk = tg.Plan(tg.Grid("ball", self.n), [(1.0, P["delta"])], react, pb, tau, precision)
        self.surf = tg.Plan(tg.Grid("sphere", self.n[1:]), [(1.0, P["epsilon"])], react, ps, tau, precision)
        self.db, self.ds = workloads.bulk_surface_perturbations(self.n, seed, amplitude)
        if not kinetics:  # O(1) fields whose total mass the exchange moves around
            self.db = self.db / amplitude
            self.ds = self.ds / amplitude
        self.oracle = BS.BulkSurface(self.n, tau, kinetics=kinetics)

    def states(self):
        return (self.bulk.state_from_deviation(self.db[None]), self.surf.state_from_deviation(self.ds[None]))

    def oracle_start(self):
        rb, rs = self.bulk.reference[0], self.surf.reference[0]
        U = [rb[q] + assemble.from_layout(self.db[q]) for q in range(2)]
        S = [rs[q] + assemble.from_layout(self.ds[q]) for q in range(2)]
        return U, S

    def full(self, plan, x):
        dev = x.double().cpu().numpy()[0]
        return dev + plan.reference[0].reshape((-1,) + (1,) * (dev.ndim - 1))

    def step(self, xb, xs):
        tg.coupled_step(self.bulk, self.surf, xb, xs, COUPLING)


def _oracle_run(pair, steps):
    U, S = pair.oracle_start()
    for _ in range(steps):
        U, S = pair.oracle.step(U, S)
    return (np.stack([assemble.to_layout(u) for u in U]), np.stack([assemble.to_layout(s) for s in S]))


@pytest.mark.parametrize("n", [(12, 20, 14), (3, 3, 3)])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 2e-7)])
@pytest.mark.parametrize("route", ["fused", "generic", "fused_stencil_apart"])
def test_coupled_steps_vs_oracle(n, precision, tol, route):
    pair = Pair(n, precision)
    pair.bulk.set_route(route)
    xb, xs = pair.states()
    steps = 10
    for _ in range(steps):
        pair.step(xb, xs)
    rb, rs = _oracle_run(pair, steps)
    eb, es = rel_err(pair.full(pair.bulk, xb), rb), rel_err(pair.full(pair.surf, xs), rs)
    # the deviations the exchange and kinetics produced, for scale
    U0, S0 = pair.oracle_start()
    moved = np.abs(rs - np.stack([assemble.to_layout(s) for s in S0])).max()
    print(n, precision, route, "bulk %.2e  surface %.2e  (surface moved %.1e)" % (eb, es, moved))
    assert eb < tol and es < tol
    assert moved > 1e-5


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_run_replays_equal_single_steps(precision):
    pair = Pair((12, 20, 14), precision)
    xb, xs = pair.states()
    yb, ys = xb.clone(), xs.clone()
    tg.coupled_run(pair.bulk, pair.surf, xb, xs, COUPLING, 19)  # two graph replays + 3 steps
    for _ in range(19):
        pair.step(yb, ys)
    assert torch.equal(xb, yb) and torch.equal(xs, ys)


def test_paper_grid_fp64():
    """(n_rho, n_theta, n_phi) = (30, 50, 30), tau = 1e-4, 20 steps."""
    pair = Pair(workloads.BULK_SURFACE["n"], "fp64", tau=workloads.BULK_SURFACE["tau"])
    xb, xs = pair.states()
    tg.coupled_run(pair.bulk, pair.surf, xb, xs, COUPLING, 20)
    rb, rs = _oracle_run(pair, 20)
    eb, es = rel_err(pair.full(pair.bulk, xb), rb), rel_err(pair.full(pair.surf, xs), rs)
    print("30x50x30 fp64: bulk %.2e  surface %.2e" % (eb, es))
    assert eb < 1e-12 and es < 1e-12


def _left_null(A):
    w = null_space(A.T)[:, 0]
    return w / w.sum()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-13), ("fp32", 1e-5)])
def test_exchange_conserves_mass(precision, tol):
    """No kinetics: sum(omega_B u) + sum(omega_S r) is invariant, with omega
    the left null vectors of the two Laplacians and the surface weight
    kappa * omega_rho[n] (the oracle pins the same identity)."""
    n = workloads.BULK_SURFACE["n"]
    # the exchange is explicit: tau kappa zeta1 eta2 (1.7 at 1e-4) must stay below 2
    pair = Pair(n, precision, tau=1e-4, kinetics=False)
    xb, xs = pair.states()
    w_rho = _left_null(op.A_rho(n[0], 3))
    w_phi = _left_null(op.A_phi(n[2]))
    w_th = np.ones(n[1]) / n[1]
    wb = np.einsum("k,j,i->kji", w_phi, w_th, w_rho)
    ws = BS.kappa(n[0]) * w_rho[-1] * np.einsum("k,j->kj", w_phi, w_th)

    def totals():
        fb, fs = pair.full(pair.bulk, xb), pair.full(pair.surf, xs)
        tot = np.array([np.sum(wb * fb[q]) + np.sum(ws * fs[q]) for q in range(2)])
        size = np.array([np.sum(wb * np.abs(fb[q])) + np.sum(ws * np.abs(fs[q])) for q in range(2)])
        return tot, size, fs

    t0, size, s0 = totals()
    tg.coupled_run(pair.bulk, pair.surf, xb, xs, COUPLING, 40)
    t1, _, s1 = totals()
    moved = np.abs(s1 - s0).max()
    print(precision, "totals", t0, "drift", t1 - t0, "surface moved %.2e" % moved)
    # the fields are N(0, 1): drift relative to sum(omega |f|)
    assert (np.abs(t1 - t0) < tol * size).all()
    assert moved > 1e-3 and np.isfinite(s1).all() and np.abs(s1).max() < 10.0


def test_batch_of_two_instances():
    """Two instances per plan (different initial data): instance b of the
    ball exchanges with instance b of the sphere only."""
    n = (8, 10, 9)
    pb = (P["alpha2"], P["beta1"], P["alpha1"])
    ps = (P["alpha2"], P["beta1"], P["zeta1"])
    bulk = tg.Plan(tg.Grid("ball", n), [(1.0, P["delta"])], "schnakenberg_scaled", pb, 1e-4, "fp64", batch=2)
    surf = tg.Plan(tg.Grid("sphere", n[1:]), [(1.0, P["epsilon"])], "schnakenberg_scaled", ps, 1e-4, "fp64",
                   batch=2)
    draws = [workloads.bulk_surface_perturbations(n, 20 + b) for b in range(2)]
    xb = bulk.state_from_deviation(np.stack([d[0] for d in draws]))
    xs = surf.state_from_deviation(np.stack([d[1] for d in draws]))
    tg.coupled_run(bulk, surf, xb, xs, COUPLING, 6)
    oracle = BS.BulkSurface(n, 1e-4)
    fb = xb.double().cpu().numpy() + bulk.reference[:, :, None, None, None]
    fs = xs.double().cpu().numpy() + surf.reference[:, :, None, None]
    for b in range(2):
        U = [bulk.reference[b, q] + assemble.from_layout(draws[b][0][q]) for q in range(2)]
        S = [surf.reference[b, q] + assemble.from_layout(draws[b][1][q]) for q in range(2)]
        for _ in range(6):
            U, S = oracle.step(U, S)
        rb = np.stack([assemble.to_layout(u) for u in U])
        rs = np.stack([assemble.to_layout(v) for v in S])
        assert rel_err(fb[b], rb) < 1e-12 and rel_err(fs[b], rs) < 1e-12, b


def test_mismatched_plans_are_rejected():
    pair = Pair((6, 8, 7), "fp64")
    xb, xs = pair.states()
    wrong = tg.Plan(tg.Grid("sphere", (8, 9)), [(1.0, 10.0)], "schnakenberg_scaled",
                    [(0.1, 0.9, 55.0)], 1e-4, "fp64")
    with pytest.raises(tg.TGError):
        tg.coupled_step(pair.bulk, wrong, xb, wrong.state_from_deviation(np.zeros((1, 2, 9, 8))), COUPLING)
    with pytest.raises(tg.TGError):
        tg.coupled_step(pair.surf, pair.bulk, xs, xb, COUPLING)
