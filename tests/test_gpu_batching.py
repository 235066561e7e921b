"""Batched and grouped runs (plans on grids of different sizes stepped by
shared persistent launches) and the autotuner, against the FP64 oracle."""
import numpy as np
import pytest

import paper_2604_11558_amd as tg
import workloads
from gpu_helpers import EPS, Case, rel_err
from oracle import assemble, reactions, splitee

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 2e-7}
# FP32 on the 256 x 512 sphere with d_v up to 40: the F tile is rounded to
# FP32 before the products, and next to the poles d sin^-2(phi) A_theta W
# is ~1e6 times the state's variation; that rounding reaches the state
# through the theta-mean mode, which phi_1 does not damp (measured 3.4e-7
# to 8.2e-7 after two steps on the instances checked).
C4_FP32_TOL = 2e-6


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_group_of_mixed_grids_matches_oracle(precision):
    """Three sphere batches of different sizes in one group: each fused
    launch of a step covers the tiles of all three plans (their theta
    contractions need different unrolled variants, so the runtime-K one
    serves all)."""
    cases = [Case("sphere", (70, 45), precision, tau=1e-2, seed=12, batch=3,
                  params=[(0.1, 0.9), (0.15, 0.8), (0.06, 1.05)],
                  diff=[(1.0, 20.0), (1.0, 12.0), (1.0, 35.0)]),
             Case("sphere", (24, 20), precision, tau=1e-2, seed=13),
             Case("sphere", (33, 40), precision, tau=1e-2, seed=11, batch=2)]
    plans = [c.plan for c in cases]
    states = [c.device_state() for c in cases]
    info = tg.group_info(plans, states)
    assert info == {"grouped": True, "launches_per_step": 2}
    tg.group_run(plans, states, 11)  # one graph replay plus 3 direct steps
    for c, x in zip(cases, states):
        err = rel_err(c.full_from_device(x), c.oracle_run(11))
        assert err < TOL[precision], (c.geometry, c.n, err)


def test_group_of_disks_one_product_launch_per_step():
    """Disks run the split products in one launch (theta sandwich plus the
    rho product and the update in the plane tail), after a stencil launch
    per plan (the plane launch updates the states in place, which the
    two-species reaction must not see); grouped, one product launch covers
    both plans."""
    cases = [Case("disk", (37, 70), "fp64", tau=1e-2, seed=19, batch=2),
             Case("disk", (32, 64), "fp64", tau=1e-2, seed=20)]
    plans = [c.plan for c in cases]
    states = [c.device_state() for c in cases]
    assert tg.group_info(plans, states) == {"grouped": True, "launches_per_step": 1 + len(plans)}
    tg.group_run(plans, states, 8)
    for c, x in zip(cases, states):
        assert rel_err(c.full_from_device(x), c.oracle_run(8)) < 1e-12


def test_group_with_stencil_apart_route():
    cases = [Case("ball", (20, 24, 37), "fp64", tau=5e-3, seed=14),
             Case("ball", (12, 16, 20), "fp64", tau=5e-3, seed=15, batch=2)]
    for c in cases:
        c.plan.set_route("fused_stencil_apart")
    plans = [c.plan for c in cases]
    states = [c.device_state() for c in cases]
    info = tg.group_info(plans, states)
    assert info["grouped"] and info["launches_per_step"] == len(plans[0].chain()) + 2
    tg.group_run(plans, states, 4)
    for c, x in zip(cases, states):
        assert rel_err(c.full_from_device(x), c.oracle_run(4)) < 1e-12


def test_group_of_split_bf16_plans_runs_member_launches():
    """Split-bf16 plans are not grouped; their launches follow each other in
    one graph and give exactly the plans' own results."""
    cases = [Case("cylinder", (27, 30, 19), "bf16x3", tau=2e-3, n_species=3, seed=16),
             Case("cylinder", (12, 10, 9), "bf16x3", tau=2e-3, n_species=3, seed=17)]
    plans = [c.plan for c in cases]
    states = [c.device_state() for c in cases]
    solo = [c.device_state() for c in cases]
    assert not tg.group_info(plans, states)["grouped"]
    tg.group_run(plans, states, 9)
    for p, x in zip(plans, solo):
        p.run(x, 9)
    for a, b in zip(states, solo):
        assert torch.equal(a, b)


@pytest.mark.parametrize("route,wide", [("fused", False), ("fused_stencil_apart", True)])
def test_c4_sphere_batches_grouped_subset_vs_oracle(route, wide):
    """64 instances on 256 x 512 and 32 on 128 x 256 with per-instance
    (a, b, d_v), FP32, grouped; 8 instances (both sizes) checked against
    the oracle after 2 steps, all instances checked finite.  Both the
    fused grouping and the one the group autotuner picks for this batch:
    F in a launch of its own and the phi product on 32-wide column tiles."""
    big, small = workloads.WORKLOADS["sphere_256x512"], workloads.WORKLOADS["sphere_128x256"]
    prm = workloads.sphere_batch_params(big.batch + small.batch)
    members = []
    for w, rows in ((big, prm[:big.batch]), (small, prm[big.batch:])):
        grid = tg.Grid("sphere", w.n)
        diff = np.stack([np.ones(w.batch), rows[:, 2]], axis=1)
        plan = tg.Plan(grid, diff, "schnakenberg", rows[:, :2], w.tau, "fp32", w.batch)
        plan.set_route(route)
        if wide:
            plan.set_tiles([32] + plan.tiles()[1:])
        pert = workloads.batch_perturbations(w)
        members.append((w, plan, pert, diff, rows))
    plans = [m[1] for m in members]
    states = [m[1].state_from_deviation(m[2]) for m in members]
    assert tg.group_info(plans, states) == {"grouped": True, "launches_per_step": 2 if route == "fused" else 4}
    steps = 2
    tg.group_run(plans, states, steps)
    for (w, plan, pert, diff, rows), x in zip(members, states):
        got = x.double().cpu().numpy()
        assert np.isfinite(got).all()
        for b in (0, 1, w.batch // 2, w.batch - 1):
            eq = reactions.equilibrium("schnakenberg", tuple(rows[b, :2]))
            W = [eq[s] + assemble.from_layout(pert[b, s]) for s in range(2)]
            se = splitee.SplitEE("sphere", w.n, diff[b], w.tau)
            react = lambda U, b=b: reactions.reaction("schnakenberg", U, tuple(rows[b, :2]))  # noqa
            for _ in range(steps):
                W = se.step(W, react)
            ref = np.stack([assemble.to_layout(u) for u in W])
            full = got[b] + plan.reference[b][:, None, None]
            err = rel_err(full, ref)
            print(w.name, b, "rel err %.2e" % err)
            assert err < C4_FP32_TOL, (w.name, b, err)


@pytest.mark.parametrize("geometry,n,precision", [("ball", (20, 24, 37), "fp64"),
                                                  ("disk", (37, 70), "fp32"),
                                                  ("cylinder", (27, 30, 19), "bf16x2")])
def test_autotune_keeps_results(geometry, n, precision):
    ns = 3 if geometry == "cylinder" else 2
    case = Case(geometry, n, precision, tau=5e-3, seed=18, n_species=ns)
    x = case.device_state()
    before = x.clone()
    res = case.plan.autotune(x, iters=3)
    assert torch.equal(x, before)  # the state is not touched
    assert np.isfinite(res["us_per_step"]) and res["us_per_step"] > 0
    assert res["route"] in tg.ROUTES
    if precision.startswith("bf16"):
        assert res["route"] != "generic"
    case.plan.run(x, 5)
    tol = {"fp64": 1e-12, "fp32": 2e-7, "bf16x2": 1.5e-6}[precision]
    assert rel_err(case.full_from_device(x), case.oracle_run(5)) < tol


def test_run_timed_matches_steps_and_counts_launches():
    case = Case("ball", (20, 24, 37), "fp32", tau=5e-3, seed=21)
    for route in ("fused", "fused_stencil_apart", "generic"):
        case.plan.set_route(route)
        x, y = case.device_state(), case.device_state()
        us = case.plan.run_timed(x, 5)
        for _ in range(5):
            case.plan.step(y)
        torch.cuda.synchronize()
        assert torch.equal(x, y)
        extra = 0 if route == "fused" else 1
        assert len(us) == len(case.plan.chain()) + extra
        assert all(u > 0 for u in us)


def test_set_tiles_checks_and_keeps_results():
    case = Case("sphere", (70, 45), "fp64", tau=1e-2, seed=22)
    tiles = case.plan.tiles()
    strided = [k for k, t in enumerate(tiles) if t in (16, 32)]
    new = list(tiles)
    for k in strided:
        new[k] = 16 if tiles[k] == 32 else 32
    case.plan.set_tiles(new)
    assert case.plan.tiles() == new
    with pytest.raises(tg.TGError):
        case.plan.set_tiles([24] * len(tiles))
    assert case.plan.tiles() == new  # unchanged by the rejected call
    x = case.device_state()
    case.plan.run(x, 6)
    assert rel_err(case.full_from_device(x), case.oracle_run(6)) < 1e-12


def test_stencil_apart_route_takes_wider_tiles():
    """On the stencil-apart route the first product has no stencil in its
    tile load, so it takes column widths whose LDS the fused route's
    in-tile stencil would overflow (the 256 x 512 sphere's 512-long phi
    contraction at 32 columns); back on the fused route the tile falls back
    to 16 columns.  Every configuration gives the same states as the
    16-wide stencil-apart one to FP32 rounding, and the oracle's to the
    FP32 bound of the 256 x 512 sphere batch."""
    case = Case("sphere", (256, 512), "fp32", tau=1e-2, seed=25)
    plan = case.plan
    tiles = plan.tiles()
    assert tiles[0] == 16
    wide = [32] + tiles[1:]
    with pytest.raises(tg.TGError):
        plan.set_tiles(wide)  # fused route: the stencil's LDS does not fit
    assert plan.tiles() == tiles
    plan.set_route("fused_stencil_apart")
    x16 = case.device_state()
    plan.run(x16, 3)
    ref = case.oracle_run(3)
    f16 = case.full_from_device(x16)
    assert rel_err(f16, ref) < C4_FP32_TOL
    plan.set_tiles(wide)
    assert plan.tiles() == wide
    x32 = case.device_state()
    plan.run(x32, 3)
    f32 = case.full_from_device(x32)
    assert rel_err(f32, ref) < C4_FP32_TOL
    assert rel_err(f32, f16) < 2.0 ** -20
    plan.set_route("fused")
    assert plan.tiles() == tiles  # back to a width the in-tile stencil fits
    x = case.device_state()
    plan.run(x, 3)
    assert rel_err(case.full_from_device(x), ref) < C4_FP32_TOL


def test_group_autotune_keeps_plans_groupable():
    cases = [Case("sphere", (70, 45), "fp32", tau=1e-2, seed=23, batch=2),
             Case("sphere", (24, 20), "fp32", tau=1e-2, seed=24)]
    plans = [c.plan for c in cases]
    states = [c.device_state() for c in cases]
    before = [s.clone() for s in states]
    us = tg.group_autotune(plans, states, iters=3)
    assert us > 0
    for a, b in zip(states, before):
        assert torch.equal(a, b)  # the states are not touched
    assert plans[0].route == plans[1].route
    assert tg.group_info(plans, states)["grouped"]
    tg.group_run(plans, states, 5)
    for c, x in zip(cases, states):
        assert rel_err(c.full_from_device(x), c.oracle_run(5)) < TOL["fp32"]


def fp64_pole_tol(case, steps):
    """FP64 steps against the oracle, relative to max|W|.  F = d M W_dev +
    g(W) is rounded where the rows of d M reach d_max ||M||_inf (the
    sin^-2 rows next to the poles: 7.1e8 on the 256 x 512 sphere), so each
    step's update carries about eps tau d_max ||M||_inf max|W_dev| from
    either side; the factor 4 as for the adjoint's bound."""
    Minf = float(abs(case.oracles[0].M).sum(axis=1).max())
    wmax = max(float(np.abs(np.asarray(e)).max()) for e in case.eq)
    dev = float(np.abs(case.pert).max()) / wmax
    return 4.0 * steps * EPS["fp64"] * (1.0 + case.tau * float(case.diff.max()) * Minf * dev)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_group_autotune_on_long_phi_contractions(precision):
    """Group autotuner on 256 x 512 and 128 x 256 spheres.  FP32: the
    stencil-apart route may widen the phi product to 32 columns; the
    states are untouched, the plans stay grouped, every tile width fits
    the chosen route (the other route can be set and set back), and the
    grouped steps match the oracle.  FP64: the 512-row phi tiles do not fit
    in LDS, so the plans have no fused route and the autotuner leaves them
    on the per-mode route (best time 0); their steps match the oracle."""
    cases = [Case("sphere", (256, 512), precision, tau=1e-2, seed=26, batch=2,
                  params=[(0.1, 0.9), (0.12, 0.85)], diff=[(1.0, 20.0), (1.0, 30.0)]),
             Case("sphere", (128, 256), precision, tau=1e-2, seed=27)]
    plans = [c.plan for c in cases]
    states = [c.device_state() for c in cases]
    before = [x.clone() for x in states]
    us = tg.group_autotune(plans, states, iters=3)
    for a, b in zip(states, before):
        assert torch.equal(a, b)
    route = plans[0].route
    print(precision, route, us, [p.tiles() for p in plans])
    if precision == "fp64":
        assert us == 0.0 and plans[0].route == "generic"
    else:
        assert us > 0
        assert all(p.route == route for p in plans)
        assert tg.group_info(plans, states)["grouped"]
        tiles = [p.tiles() for p in plans]
        other = "fused" if route == "fused_stencil_apart" else "fused_stencil_apart"
        for p, t in zip(plans, tiles):
            p.set_route(other)
            p.set_route(route)
            if route == "fused":
                assert p.tiles() == t  # route 0's widths survive the round trip
        for p, t in zip(plans, tiles):
            p.set_tiles(t)  # the autotuner's widths are valid for its route
    tg.group_run(plans, states, 2)
    for c, x in zip(cases, states):
        tol = fp64_pole_tol(c, 2) if precision == "fp64" else C4_FP32_TOL
        err = rel_err(c.full_from_device(x), c.oracle_run(2))
        print(c.n, "rel err %.2e (bound %.2e)" % (err, tol))
        assert err < tol


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_disk_plane_launch_with_more_workgroups_than_fit(precision):
    """The disk's fused step runs one plane launch per (instance, species)
    that updates the state in place, and the reaction of each species reads
    the other species' state.  With 2048 identical instances there are more
    workgroups than the GPU holds at once, so the two species' workgroups of
    an instance can start far apart: F is computed by a launch of its own
    first, every instance matches the oracle, and all are bit-identical."""
    B = 2048
    one = Case("disk", (32, 64), precision, tau=1e-2, seed=31, amplitude=1e-3)
    plan = tg.Plan(one.grid, np.repeat(one.diff, B, axis=0), one.kind, np.repeat(one.params, B, axis=0),
                   one.tau, precision, B)
    assert plan.route == "fused"
    x = plan.state_from_deviation(np.repeat(one.pert, B, axis=0))
    assert len(plan.run_timed(x.clone(), 1)) == len(plan.chain()) + 1  # the stencil launch first
    plan.run(x, 4)
    dev = x.detach().double().cpu().numpy().reshape((B, 2, 64, 32))
    assert np.array_equal(dev, np.repeat(dev[:1], B, axis=0))
    ref = one.oracle_run(4)[0]
    got = dev[0] + plan.reference[0][:, None, None]
    assert rel_err(got, ref) < TOL[precision]
