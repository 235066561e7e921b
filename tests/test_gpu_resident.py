"""Route 4 (resident steps) on the disk: one workgroup per instance keeps the
state, F and the sandwich intermediate of every species in LDS and runs many
split steps per launch.  Checked against the FP64 oracle (element by
element, several tiles and ragged edges), against the fused route, across
the 1024-step launch chunks, with per-instance parameters and a batch larger
than the GPU holds at once, plus the route's refusals and its error paths."""
import numpy as np
import pytest

import paper_2604_11558_amd as tg
from gpu_helpers import Case, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 2e-7}

# (geometry, grid, precisions whose tiles fit in LDS): 32 x 64 is the small
# disk workload; 37 x 70 and 20 x 27 leave ragged 16-wide tiles; 3 x 3 is
# the smallest grid.  37 x 70 in FP64 does not fit (checked below).
GRIDS = [("disk", (32, 64), ("fp64", "fp32")), ("disk", (20, 27), ("fp64", "fp32")),
         ("disk", (3, 3), ("fp64", "fp32")), ("disk", (37, 70), ("fp32",)),
         ("disk_lambda", (32, 64), ("fp64", "fp32")), ("disk_lambda", (37, 70), ("fp32",))]
CASES = [(g, n, p) for g, n, ps in GRIDS for p in ps]


@pytest.mark.parametrize("geometry,n,precision", CASES)
def test_resident_run_matches_oracle(geometry, n, precision):
    case = Case(geometry, n, precision, tau=1e-2, seed=41)
    case.plan.set_route("resident")
    assert case.plan.route == "resident"
    assert len(case.plan.chain()) == 1
    x = case.device_state()
    case.plan.run(x, 12)                     # one launch of 12 steps
    err = rel_err(case.full_from_device(x), case.oracle_run(12))
    print(geometry, n, precision, "resident vs oracle %.2e" % err)
    assert err < TOL[precision]


# the general form (factors from L2, phi_1 per step): 40 x 48 is wider than
# the 64 x 32 register-resident tiles in both precisions; three species
# (the cubic activator-inhibitor-substrate kinetics) always take it.
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_general_form_matches_oracle(precision):
    case = Case("disk", (40, 48), precision, tau=1e-2, seed=52)
    case.plan.set_route("resident")
    x = case.device_state()
    case.plan.run(x, 9)
    err = rel_err(case.full_from_device(x), case.oracle_run(9))
    print("disk (40, 48)", precision, "general resident vs oracle %.2e" % err)
    assert err < TOL[precision]


def test_three_species_matches_oracle():
    case = Case("disk", (32, 64), "fp32", tau=5e-3, seed=53, n_species=3)
    case.plan.set_route("resident")
    x = case.device_state()
    case.plan.run(x, 9)
    err = rel_err(case.full_from_device(x), case.oracle_run(9))
    print("disk (32, 64) 3 species fp32 resident vs oracle %.2e" % err)
    assert err < TOL["fp32"]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_single_steps_equal_one_multi_step_launch(precision):
    case = Case("disk", (32, 64), precision, tau=1e-2, seed=42)
    case.plan.set_route("resident")
    x = case.device_state()
    y = x.clone()
    case.plan.run(x, 7)
    for _ in range(7):
        case.plan.step(y)
    # the same arithmetic in the same order: bit for bit
    assert torch.equal(x, y)
    assert len(case.plan.run_timed(y.clone(), 2)) == 1


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_resident_equals_fused_route_across_chunks(precision):
    """1030 steps: a 1024-step launch and a 6-step one, against the fused
    route's graph replays (the same step, arithmetic in another order)."""
    case = Case("disk", (32, 64), precision, tau=1e-3, seed=43, amplitude=1e-2)
    x = case.device_state()
    y = x.clone()
    case.plan.set_route("resident")
    case.plan.run(x, 1030)
    case.plan.set_route("fused")
    case.plan.run(y, 1030)
    err = rel_err(case.full_from_device(x), case.full_from_device(y))
    print(precision, "resident vs fused after 1030 steps %.2e" % err)
    assert err < {"fp64": 1e-12, "fp32": 1e-5}[precision]


def test_batch_with_per_instance_parameters():
    params = [(0.1, 0.9), (0.15, 0.8), (0.06, 1.05)]
    diff = [(1.0, 20.0), (1.0, 12.0), (1.0, 35.0)]
    case = Case("disk", (32, 64), "fp64", tau=1e-2, seed=44, batch=3, params=params, diff=diff)
    case.plan.set_route("resident")
    x = case.device_state()
    case.plan.run(x, 9)
    assert rel_err(case.full_from_device(x), case.oracle_run(9)) < 1e-12


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_more_instances_than_fit(precision):
    """2048 identical instances (more workgroups than the GPU holds at once):
    every instance equals the first bit for bit and matches the oracle."""
    B = 2048
    one = Case("disk", (32, 64), precision, tau=1e-2, seed=45)
    plan = tg.Plan(one.grid, np.repeat(one.diff, B, axis=0), one.kind, np.repeat(one.params, B, axis=0),
                   one.tau, precision, B)
    plan.set_route("resident")
    x = plan.state_from_deviation(np.repeat(one.pert, B, axis=0))
    plan.run(x, 5)
    dev = x.detach().double().cpu().numpy().reshape((B, 2, 64, 32))
    assert np.array_equal(dev, np.repeat(dev[:1], B, axis=0))
    got = dev[0] + plan.reference[0][:, None, None]
    assert rel_err(got, one.oracle_run(5)[0]) < TOL[precision]


def test_indicators_on_the_resident_route():
    """run_diag keeps route 4 for the plain steps and takes the fused
    launches for the recorded ones: the same records and state as route 0."""
    case = Case("disk", (32, 64), "fp64", tau=1e-2, seed=46, amplitude=1e-2)
    x = case.device_state()
    y = x.clone()
    case.plan.set_route("resident")
    rx = case.plan.run_diag(x, 23, every=5).cpu().numpy()
    case.plan.set_route("fused")
    ry = case.plan.run_diag(y, 23, every=5).cpu().numpy()
    assert rx.shape == ry.shape == (4, 1, 2, 2)
    assert np.abs(rx - ry).max() <= 1e-12 * np.abs(ry).max()
    assert rel_err(case.full_from_device(x), case.full_from_device(y)) < 1e-12


def test_routes_that_do_not_apply_are_refused():
    for geometry, n, precision in (("sphere", (24, 20), "fp64"), ("ball", (8, 10, 12), "fp32"),
                                   ("disk", (37, 70), "fp64"), ("disk", (12, 16), "bf16x3")):
        case = Case(geometry, n, precision, seed=47)
        before = case.plan.route
        with pytest.raises(tg.TGError):
            case.plan.set_route("resident")
        assert case.plan.route == before


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_non_finite_state_is_reported(precision):
    case = Case("disk", (32, 64), precision, seed=48)
    case.plan.set_route("resident")
    x = case.device_state()
    x.view(-1)[100] = float("nan")
    with pytest.raises(tg.TGError) as ei:
        case.plan.run(x, 3)
    assert "non-finite" in str(ei.value)
    z = case.device_state()
    case.plan.run(z, 3)          # the flag was cleared
    assert torch.isfinite(z).all()


def test_autotune_keeps_parity():
    case = Case("disk", (32, 64), "fp32", tau=1e-2, seed=49)
    x = case.device_state()
    res = case.plan.autotune(x, iters=5)
    print("autotuned", res, case.plan.route)
    case.plan.run(x, 6)
    assert rel_err(case.full_from_device(x), case.oracle_run(6)) < TOL["fp32"]


def test_group_run_with_a_resident_member():
    """A resident disk plan grouped with a sphere plan: each member runs its
    steps as tg_run would, and both match the oracle."""
    disk = Case("disk", (32, 64), "fp64", tau=1e-2, seed=50, batch=2,
                params=[(0.1, 0.9), (0.15, 0.8)], diff=[(1.0, 20.0), (1.0, 12.0)])
    sph = Case("sphere", (24, 20), "fp64", tau=1e-2, seed=51)
    disk.plan.set_route("resident")
    states = [disk.device_state(), sph.device_state()]
    info = tg.group_info([disk.plan, sph.plan], states)
    assert not info["grouped"]
    tg.group_run([disk.plan, sph.plan], states, 11)
    assert rel_err(disk.full_from_device(states[0]), disk.oracle_run(11)) < 1e-12
    assert rel_err(sph.full_from_device(states[1]), sph.oracle_run(11)) < 1e-12


@pytest.mark.parametrize("precision,B", [("fp64", 600), ("fp32", 1000)])
def test_resident_route_just_past_one_round_of_plane_workgroups(precision, B):
    """Batches whose plane launch takes a little more than one round of
    workgroups (FP64: 40 KB of LDS each, 4 per CU, 1024 on 256 CUs, so 600
    instances of two species give 1200; FP32: 22 KB, 7 per CU, 1792, so 1000
    give 2000) keep the plane launch, so the resident route stays offered."""
    one = Case("disk", (32, 64), precision, tau=1e-2, seed=46)
    plan = tg.Plan(one.grid, np.repeat(one.diff, B, axis=0), one.kind, np.repeat(one.params, B, axis=0),
                   one.tau, precision, B)
    plan.set_route("resident")
    assert plan.route == "resident"
    x = plan.state_from_deviation(np.repeat(one.pert, B, axis=0))
    plan.run(x, 3)
    dev = x.detach().double().cpu().numpy().reshape((B, 2, 64, 32))
    got = dev[B - 1] + plan.reference[B - 1][:, None, None]
    assert rel_err(got, one.oracle_run(3)[0]) < TOL[precision]
