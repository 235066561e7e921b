"""Steady-state indicators (integral mean, L2 norm of a step's increment),
gathered in the update epilogue of every route and precision, against

* the FP64 oracle stepping the same problem (oracle weights and states);
* the same formulas in NumPy on the device's own old and new states, which
  isolates the fused reduction from the precision of the step;

plus: the state after a step with indicators equals the plain step's bit for
bit, records of `run_diag` equal `run`'s state, and repeated calls give
identical indicators (no atomics in the sums)."""
import math

import numpy as np
import pytest

from gpu_helpers import Case
from oracle import diagnostics as D

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GRIDS = [("disk", (37, 70), 2), ("sphere", (70, 45), 2), ("ball", (20, 24, 37), 2),
         ("cylinder", (27, 30, 19), 3), ("disk_lambda", (37, 70), 2), ("disk", (3, 3), 2),
         ("ball", (3, 3, 3), 2)]


def _weights(case):
    return D.weights(case.geometry, case.n, case.extent)


def _layout(w):
    """[i, j(, k)] -> the device layout [k][j][i]."""
    return np.ascontiguousarray(w.T)


def _numpy_indicators(case, old_dev, new_dev):
    """The indicators from the device's own deviation states (float64 math)."""
    w = _layout(_weights(case))
    ref = case.plan.reference
    out = np.empty((case.batch, case.ns, 2))
    for b in range(case.batch):
        for s in range(case.ns):
            o = old_dev[b, s].astype(np.float64)
            n = new_dev[b, s].astype(np.float64)
            out[b, s, 0] = ref[b, s] + np.sum(w * n) / np.sum(w)
            out[b, s, 1] = math.sqrt(np.sum(w * (n - o) ** 2))
    return out


def _dev(case, x):
    return x.detach().cpu().numpy().reshape((case.batch, case.ns) + tuple(reversed(case.n)))


@pytest.mark.parametrize("geometry,n,ns", GRIDS)
@pytest.mark.parametrize("route", ["fused", "generic", "fused_stencil_apart"])
def test_step_diag_vs_oracle_fp64(geometry, n, ns, route):
    case = Case(geometry, n, "fp64", tau=5e-3, n_species=ns, seed=7, amplitude=1e-2)
    case.plan.set_route(route)
    x = case.device_state()
    W0 = case.oracle_full(0)
    diag = case.plan.step_diag(x).cpu().numpy()[0]
    W1 = case.oracle_run(1)[0]
    w = _weights(case)
    from oracle import assemble
    vol = float(np.sum(w))
    for s in range(ns):
        U1 = assemble.from_layout(W1[s])
        mean = D.integral_mean(U1, w)
        inc = D.increment_norm(U1, W0[s], w)
        big = max(np.abs(U1).max(), np.abs(W0[s]).max())
        print(geometry, n, route, s, "mean %.3e (%.1e)  inc %.3e (%.1e)" %
              (mean, diag[s, 0] - mean, inc, diag[s, 1] - inc))
        # the states agree to 1e-12 max|W|; so do their weighted sums
        assert abs(diag[s, 0] - mean) <= 1e-12 * big
        assert abs(diag[s, 1] - inc) <= 1e-12 * big * math.sqrt(vol)
        assert inc > 0.0


@pytest.mark.parametrize("geometry,n,ns", GRIDS[:5])
@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x2", "bf16x3"])
@pytest.mark.parametrize("route", ["fused", "generic", "fused_stencil_apart"])
def test_fused_reduction_matches_numpy_on_device_states(geometry, n, ns, precision, route):
    if precision.startswith("bf16") and route == "generic":
        pytest.skip("split-bf16 plans run the fused routes only")
    case = Case(geometry, n, precision, tau=5e-3, n_species=ns, seed=8, amplitude=1e-2)
    case.plan.set_route(route)
    x = case.device_state()
    y = x.clone()
    old = _dev(case, x)
    diag = case.plan.step_diag(x).cpu().numpy()
    case.plan.step(y)
    assert torch.equal(x, y), "the indicators changed the step"
    ref = _numpy_indicators(case, old, _dev(case, x))
    err_m = np.abs(diag[..., 0] - ref[..., 0]).max() / np.abs(ref[..., 0]).max()
    err_i = np.abs(diag[..., 1] - ref[..., 1]).max() / np.abs(ref[..., 1]).max()
    print(geometry, n, precision, route, "mean %.1e  inc %.1e" % (err_m, err_i))
    assert err_m < 1e-13 and err_i < 1e-12


def test_batch_slabs_and_reproducibility():
    params = [(0.1, 0.9), (0.15, 0.8), (0.06, 1.05)]
    diff = [(1.0, 20.0), (1.0, 12.0), (1.0, 35.0)]
    case = Case("sphere", (40, 33), "fp32", tau=1e-2, seed=5, batch=3, params=params, diff=diff,
                amplitude=1e-2)
    x = case.device_state()
    x2 = x.clone()
    old = _dev(case, x)
    d1 = case.plan.step_diag(x).cpu().numpy()
    d2 = case.plan.step_diag(x2).cpu().numpy()
    assert np.array_equal(d1, d2)
    ref = _numpy_indicators(case, old, _dev(case, x))
    assert np.abs(d1 - ref).max() / np.abs(ref).max() < 1e-12
    # instances differ, so a mix-up of slabs would show
    assert len({round(v, 12) for v in d1[:, 1, 1]}) == 3


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_run_diag_records_and_state(precision):
    case = Case("disk", (37, 70), precision, tau=5e-3, seed=9, amplitude=1e-2)
    x = case.device_state()
    y = x.clone()
    z = x.clone()
    rec = case.plan.run_diag(x, 21, every=4).cpu().numpy()   # records after steps 4, 8, ..., 20
    case.plan.run(y, 21)
    assert rec.shape == (5, 1, 2, 2)
    assert torch.equal(x, y)
    # fewer steps than one record: plain steps, an empty record buffer
    x2, y2 = x.clone(), x.clone()
    assert case.plan.run_diag(x2, 3, every=4).shape[0] == 0
    case.plan.run(y2, 3)
    assert torch.equal(x2, y2)
    for r in range(5):
        case.plan.run(z, 3)
        old = _dev(case, z)
        d = case.plan.step_diag(z).cpu().numpy()
        assert np.array_equal(d, rec[r]), r
        ref = _numpy_indicators(case, old, _dev(case, z))
        assert np.abs(d - ref).max() / np.abs(ref).max() < 1e-12


def test_full_size_ball_fp32_fused():
    """The 64 x 64 x 128 ball in the benchmark's launch configuration."""
    case = Case("ball", (64, 64, 128), "fp32", tau=5e-3, seed=3)
    assert case.plan.route == "fused"
    x = case.device_state()
    old = _dev(case, x)
    d = case.plan.step_diag(x).cpu().numpy()
    ref = _numpy_indicators(case, old, _dev(case, x))
    err = np.abs(d - ref).max() / np.abs(ref).max()
    print("ball 64x64x128 fp32 indicators", d[0], "err %.1e" % err)
    assert err < 1e-12
