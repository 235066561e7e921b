"""Edge cases of the device entry points: zero steps leave every state bit
for bit unchanged, a non-finite value raised by an update is reported (and
the flag cleared for the next run), misaligned or mismatched buffers are
refused before any launch."""
import numpy as np
import pytest

import paper_2604_11558_amd as tg
from gpu_helpers import Case
from oracle import bulk_surface as BS

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("geometry,n", [("disk", (12, 16)), ("ball", (8, 10, 12))])
def test_zero_steps_change_nothing(geometry, n):
    case = Case(geometry, n, "fp32", seed=2)
    x = case.device_state()
    y = x.clone()
    case.plan.run(x, 0)
    assert torch.equal(x, y)
    assert case.plan.run_diag(x, 0, every=1).shape[0] == 0
    assert torch.equal(x, y)
    tg.group_run([case.plan], [x], 0)
    assert torch.equal(x, y)


def test_zero_coupled_steps_change_nothing():
    p = BS.PARAMS
    n = (6, 8, 7)
    bulk = tg.Plan(tg.Grid("ball", n), [(1.0, 10.0)], "schnakenberg_scaled", (0.1, 0.9, 55.0), 1e-4, "fp64")
    surf = tg.Plan(tg.Grid("sphere", n[1:]), [(1.0, 10.0)], "schnakenberg_scaled", (0.1, 0.9, 55.0), 1e-4, "fp64")
    xb = bulk.state_from_deviation(1e-3 * np.ones(bulk.state_shape))
    xs = surf.state_from_deviation(1e-3 * np.ones(surf.state_shape))
    yb, ys = xb.clone(), xs.clone()
    tg.coupled_run(bulk, surf, xb, xs, (p["zeta1"], p["zeta2"], p["zeta3"], p["eta1"], p["eta2"]), 0)
    assert torch.equal(xb, yb) and torch.equal(xs, ys)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_non_finite_state_is_reported_then_cleared(precision):
    case = Case("disk", (12, 16), precision, seed=3)
    x = case.device_state()
    x.view(-1)[5] = float("nan")
    with pytest.raises(tg.TGError) as ei:
        case.plan.run(x, 3)
    assert "non-finite" in str(ei.value)
    # the flag was cleared: a clean state runs again without error
    z = case.device_state()
    case.plan.run(z, 3)
    assert torch.isfinite(z).all()
    # single steps report through tg_sync_status
    y = case.device_state()
    y.view(-1)[7] = float("inf")
    case.plan.step(y)
    with pytest.raises(tg.TGError):
        case.plan.sync_status()
    case.plan.sync_status()  # cleared


def test_misaligned_and_mismatched_buffers_are_refused():
    case = Case("disk", (12, 16), "fp64", seed=4)
    x = case.device_state()
    big = torch.zeros(x.numel() + 1, dtype=x.dtype, device=x.device)
    view = big[1:]                      # contiguous, but 8 bytes off the 32-byte vector alignment
    assert view.is_contiguous() and view.numel() == x.numel()
    with pytest.raises(tg.TGError):
        case.plan.step(view)
    with pytest.raises(ValueError):
        case.plan.step(x.float())       # wrong element type
    with pytest.raises(ValueError):
        case.plan.step(x[..., :-1].contiguous())  # wrong size


def test_overlapping_operator_buffers_are_refused():
    """The stencil reads its input through a restrict-qualified pointer, so
    tg_apply_operator refuses an output that overlaps the input (TG_EINVAL)
    before any launch, and the plan still works afterwards."""
    case = Case("disk", (12, 16), "fp64", seed=4)
    x = case.device_state()
    n = x.numel()
    big = torch.zeros(2 * n, dtype=x.dtype, device=x.device)
    big[:n].copy_(x.view(-1))
    a, b = big[:n].view(x.shape), big[4:n + 4].view(x.shape)  # both 32-byte aligned
    with pytest.raises(tg.TGError) as err:
        case.plan.apply_operator(a, b)
    assert err.value.code == -1
    out = torch.empty_like(x)
    case.plan.apply_operator(x, out)
    ref = torch.empty_like(x)
    case.plan.apply_operator(x, ref)
    assert torch.equal(out, ref)


def test_oversized_plan_reports_enomem_and_the_device_stays_usable():
    """A plan whose scratch buffers exceed the device memory: 9000 instances
    of two species on a 128^3 cylinder in FP64 need two state-sized buffers
    of 302 GB each, more than the 288 GB of HBM; the first allocation fails
    without touching memory.  TG_ENOMEM, and later plans work."""
    g = tg.Grid("cylinder", (128, 128, 128))
    B = 9000
    with pytest.raises(tg.TGError) as err:
        tg.Plan(g, np.tile([1.0, 20.0], (B, 1)), "schnakenberg", np.tile([0.1, 0.9], (B, 1)), 1e-2, "fp64", B)
    assert err.value.code == -2, err.value
    small = tg.Plan(tg.Grid("disk", (8, 12)), [(1.0, 20.0)], "schnakenberg", (0.1, 0.9), 1e-2, "fp64")
    x = small.state_from_deviation(1e-3 * np.ones(small.state_shape))
    small.run(x, 3)
    assert torch.isfinite(x).all()
