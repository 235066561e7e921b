"""tg_step_diag_noalloc (indicator partial sums in the library's static
device scratch, no allocation in the call) against tg_step_diag: the same
step and the same indicators, bit for bit, on two calls in a row -- the
second on a smaller plan -- and a plan too large for the scratch is
refused with TG_EINVAL."""

import numpy as np
import pytest

import paper_2604_11558_amd as tg
from gpu_helpers import Case

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_matches_step_diag_twice_then_smaller(precision):
    """Two calls in a row on a ball plan, then two on a smaller disk batch
    (the scratch keeps the last call's contents; nothing may depend on it)."""
    big = Case("ball", (20, 24, 37), precision, tau=5e-3, seed=3)
    small = Case("disk", (13, 18), precision, tau=1e-2, seed=4, batch=2)
    for case in (big, small):
        x_ref = case.device_state()
        x_new = x_ref.clone()
        for call in range(2):
            d_ref = case.plan.step_diag(x_ref)
            d_new = torch.full((case.batch, case.ns, 2), float("nan"), dtype=torch.float64, device="cuda")
            case.plan.step_diag_noalloc(x_new, d_new)
            torch.cuda.synchronize()
            print(case.geometry, precision, call, d_new.flatten().tolist())
            assert torch.equal(x_ref, x_new), (case.geometry, call)
            assert torch.equal(d_ref, d_new), (case.geometry, call, d_ref, d_new)


def test_noalloc_matches_oracle_indicators_on_a_small_grid():
    """The records of the no-allocation call after two steps equal those of
    tg_step_diag after two steps (which the indicator tests hold to the
    oracle)."""
    case = Case("sphere", (30, 22), "fp64", tau=1e-2, seed=5)
    a, b = case.device_state(), case.device_state()
    da = case.plan.step_diag(a)
    db = torch.empty_like(da)
    case.plan.step_diag_noalloc(b, db)
    da = case.plan.step_diag(a)
    case.plan.step_diag_noalloc(b, db)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(da, db)


def test_noalloc_refuses_plans_beyond_the_scratch():
    # 2 * (npts / 8 + 64) * nslab doubles: 256 x 512 sphere with 64
    # instances of two species needs 33.7 MB > 16 MiB
    grid = tg.Grid("sphere", (256, 512))
    plan = tg.Plan(grid, [(1.0, 20.0)] * 64, "schnakenberg", [(0.1, 0.9)] * 64, 1e-2, "fp32", 64)
    x = torch.zeros(plan.state_shape, dtype=torch.float32, device="cuda")
    out = torch.empty((64, 2, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(tg.TGError) as err:
        plan.step_diag_noalloc(x, out)
    assert err.value.code == -1 and "static scratch" in str(err.value)
    assert torch.count_nonzero(x) == 0
