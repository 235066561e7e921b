"""tg_run_history: the states it keeps are the states single steps pass
through, on the fused, per-mode and resident routes."""
import numpy as np
import pytest

import paper_2604_11558_amd as tg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("geometry,n,precision,route", [
    ("disk", (37, 70), "fp64", "fused"), ("disk", (37, 70), "fp32", "generic"),
    ("ball", (12, 10, 14), "fp32", "fused_stencil_apart"), ("disk", (32, 64), "fp64", "resident")])
def test_history_slots_are_the_stepped_states(geometry, n, precision, route):
    grid = tg.Grid(geometry, n)
    plan = tg.Plan(grid, [(1.0, 20.0)], "schnakenberg", (0.1, 0.9), 1e-2, precision)
    plan.set_route(route)
    dev = 1e-2 * np.random.default_rng(4).standard_normal(plan.state_shape)
    x = plan.state_from_deviation(dev)
    y = x.clone()
    steps = 6
    hist = torch.empty((steps,) + tuple(x.shape), dtype=x.dtype, device=x.device)
    plan.run_history(x, steps, hist)
    for k in range(steps):
        assert torch.equal(hist[k], y), k
        plan.step(y)
    torch.cuda.synchronize()
    assert torch.equal(x, y)


def test_history_widened_to_fp64():
    """An FP32 plan's history kept in FP64: the stepped states, exactly widened."""
    plan = tg.Plan(tg.Grid("disk", (37, 70)), [(1.0, 20.0)], "schnakenberg", (0.1, 0.9), 1e-2, "fp32")
    x = plan.state_from_deviation(1e-2 * np.random.default_rng(5).standard_normal(plan.state_shape))
    y = x.clone()
    hist = torch.empty((5,) + tuple(x.shape), dtype=torch.float64, device=x.device)
    plan.run_history(x, 5, hist)
    for k in range(5):
        assert torch.equal(hist[k], y.double()), k
        plan.step(y)
    torch.cuda.synchronize()
    assert torch.equal(x, y)


def test_history_overlapping_the_state_is_refused():
    plan = tg.Plan(tg.Grid("disk", (16, 24)), [(1.0, 20.0)], "schnakenberg", (0.1, 0.9), 1e-2, "fp64")
    hist = torch.zeros((4,) + tuple(plan.state_shape), dtype=torch.float64, device="cuda")
    with pytest.raises(tg.TGError) as err:
        tg._check(tg.lib().tg_run_history(plan._h, hist[2].data_ptr(), 4, hist.data_ptr(), 0, None))
    assert err.value.code == -1  # TG_EINVAL, before any launch
