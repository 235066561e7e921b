"""Full-length accuracy records of the benchmark workloads.

Every workload runs its whole configured length, and the error of each
reduced-precision trajectory is recorded along the way:

* the 64 x 64 x 128 ball, 500 steps: FP64 and FP32 in lockstep with the
  FP64 oracle, the error after every step;
* the 100^3 cylinder (three species), 1000 steps: split-bf16 with two and
  three terms and FP32 against the FP64 device trajectory (itself held to
  the oracle at 1e-12), every step;
* the sphere batch, 2000 steps: eight instances covering both grid sizes
  and the parameter range, FP32 (grouped launches) against FP64 plans of
  the same instances, every 100 steps;
* the 256 x 512 disk gradient, 400 steps: FP32 forward with the
  checkpointed reverse sweep against central differences of the FP64
  device loss.

Errors are reported relative to max |W| and, where the state is a small
perturbation of an equilibrium, relative to max |W - w_ref| (the part the
steps change).
"""
import numpy as np
import pytest

import paper_2604_11558_amd as tg
import workloads
from oracle import assemble, reactions, splitee

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _full(plan, x):
    dev = x.double().cpu().numpy()
    return dev + plan.reference.reshape(plan.reference.shape + (1,) * (dev.ndim - 2))


def test_ball_500_steps_lockstep_with_oracle():
    """FP64 within 1e-12 of the oracle at every one of the 500 steps; FP32
    within its bound at every step (bounds derived in the comments).

    The oracle steps the deviation W - w_e here (its own step function with
    the reaction evaluated at w_e + deviation): the same map, since M takes
    constants to zero and the split action is linear.  Stepping full values
    instead, its own FP64 rounding of M (w_e + dev) drifts from the
    deviation form by about 3e-15 of max |W| per step (2e-12 after 500
    steps), more than the device differs from either."""
    w = workloads.WORKLOADS["ball_64x64x128"]
    grid = tg.Grid(w.geometry, w.n, w.extent)
    pert = workloads.perturbation(w)
    eq = reactions.equilibrium(w.reaction, w.params)
    p64 = tg.Plan(grid, w.diff, w.reaction, w.params, w.tau, "fp64")
    p32 = tg.Plan(grid, w.diff, w.reaction, w.params, w.tau, "fp32")
    x64 = p64.state_from_deviation(pert[None])
    x32 = p32.state_from_deviation(pert[None])
    se = splitee.make(w)
    react = lambda U: reactions.reaction(w.reaction, [eq[s] + U[s] for s in range(len(U))],  # noqa: E731
                                         w.params)
    D = [assemble.from_layout(pert[s]) for s in range(w.n_species)]
    e64, e32, e32d = [], [], []
    for it in range(w.steps):
        p64.step(x64)
        p32.step(x32)
        D = se.step(D, react)
        dev = np.stack([assemble.to_layout(u) for u in D])
        ref = dev + np.asarray(eq).reshape(-1, 1, 1, 1)
        g64, g32 = _full(p64, x64)[0], _full(p32, x32)[0]
        scale = np.abs(ref).max()
        e64.append(float(np.abs(g64 - ref).max() / scale))
        e32.append(float(np.abs(g32 - ref).max() / scale))
        e32d.append(float(np.abs(g32 - ref).max() / np.abs(dev).max()))
        if (it + 1) % 50 == 0:
            print("step %3d: fp64 %.2e  fp32 %.2e (deviation-relative %.2e, max|dev| %.2e)"
                  % (it + 1, e64[-1], e32[-1], e32d[-1], np.abs(dev).max()), flush=True)
    print("worst over %d steps: fp64 %.2e  fp32 %.2e  fp32 deviation-relative %.2e"
          % (w.steps, max(e64), max(e32), max(e32d)))
    assert max(e64) < 1e-12
    # FP32: the state is the deviation (FP32 storage, 2^-24 relative to it);
    # a step applies five products with eigenvector conditioning up to
    # sqrt(2n) = 16, so one step adds at most ~5 * 16 * 2^-24 = 4.8e-6 of
    # max|dev|; the scheme is contractive for the deviation (Turing-stable
    # kinetics), so earlier errors do not grow.  Bound: 5e-5 of max|dev|
    # (the FP32 bound of the short tests, 2e-7 of max|W|, holds as well)
    assert max(e32d) < 5e-5
    assert max(e32) < 2e-7


def _c3(precision):
    w = workloads.WORKLOADS["cylinder_100x100x100"]
    grid = tg.Grid(w.geometry, w.n, w.extent)
    plan = tg.Plan(grid, w.diff, w.reaction, w.params, w.tau, precision)
    return w, plan, plan.state_from_deviation(workloads.perturbation(w)[None])


# Regression bounds relative to max |W| over the whole run: four times the
# worst error measured on this seeded workload (bf16x2 3.3e-6, bf16x3
# 2.0e-7, FP32 9.2e-8 of max |W|; 7.4e-3, 4.4e-4, 1.6e-4 of max |W - w_ref|).
# The errors grow over the first ~600 steps and then level off as the
# deviation decays.  What dominates is not the products' operand rounding
# (that model gives ~2e-5 of max |dev| per step for FP32) but the rounding of
# F to the storage type next to the axis, where d rho^-2 A_theta W is ~1e9
# times the deviation and the theta-mean part of that rounding passes the
# theta factor undamped -- the same mechanism as at the sphere's poles.
C3_TOL = {"bf16x2": 1.5e-5, "bf16x3": 8e-7, "fp32": 4e-7}


def test_cylinder_1000_steps_reduced_precisions_vs_fp64():
    w, p64, x64 = _c3("fp64")
    others = {p: _c3(p)[1:] for p in ("bf16x2", "bf16x3", "fp32")}
    ref = torch.from_numpy(p64.reference[0]).cuda().view(-1, 1, 1, 1)
    worst = {p: [0.0, 0.0] for p in others}
    for it in range(w.steps):
        p64.step(x64)
        for p, (plan, x) in others.items():
            plan.step(x)
        if (it + 1) % 10 == 0 or it < 10:
            full64 = x64[0] + ref
            scale = float(full64.abs().max())
            dmax = float(x64.abs().max())
            for p, (plan, x) in others.items():
                diff = float((x[0].double() - x64[0]).abs().max())
                worst[p][0] = max(worst[p][0], diff / scale)
                worst[p][1] = max(worst[p][1], diff / dmax)
            if (it + 1) % 100 == 0:
                print("step %4d: max|dev| %.2e  " % (it + 1, dmax)
                      + "  ".join("%s %.2e (dev %.2e)" % (p, worst[p][0], worst[p][1]) for p in others),
                      flush=True)
    for p in others:
        print("%s worst over %d steps: %.2e of max|W| (bound %.1e), %.2e of max|dev|"
              % (p, w.steps, worst[p][0], C3_TOL[p], worst[p][1]))
        assert worst[p][0] < C3_TOL[p], (p, worst[p])


def test_sphere_batch_2000_steps_fp32_grouped_vs_fp64():
    """Eight instances of the 96-instance batch, four per grid size (first,
    last and two in between), with their own (a, b, d_v); the FP32 group
    in the configuration the group autotuner picks for the whole batch (F
    in a launch of its own, the phi product on 32-wide column tiles)."""
    big, small = workloads.WORKLOADS["sphere_256x512"], workloads.WORKLOADS["sphere_128x256"]
    prm = workloads.sphere_batch_params(big.batch + small.batch)
    pick = {big: [0, 21, 42, 63], small: [0, 10, 20, 31]}
    plans = {"fp32": [], "fp64": []}
    states = {"fp32": [], "fp64": []}
    for wl, off in ((big, 0), (small, big.batch)):
        idx = pick[wl]
        rows = prm[[off + i for i in idx]]
        diff = np.stack([np.ones(len(idx)), rows[:, 2]], axis=1)
        pert = np.stack([workloads.perturbation(wl, wl.seed + i) for i in idx])
        for prec in ("fp32", "fp64"):
            plan = tg.Plan(tg.Grid("sphere", wl.n), diff, "schnakenberg", rows[:, :2], wl.tau, prec, len(idx))
            if prec == "fp32":
                plan.set_route("fused_stencil_apart")
                plan.set_tiles([32] + plan.tiles()[1:])
            plans[prec].append(plan)
            states[prec].append(plan.state_from_deviation(pert))
    worst_w = worst_d = 0.0
    done = 0
    while done < big.steps:
        tg.group_run(plans["fp32"], states["fp32"], 100)
        tg.group_run(plans["fp64"], states["fp64"], 100)
        done += 100
        for k in range(2):
            p64, x64, x32 = plans["fp64"][k], states["fp64"][k], states["fp32"][k]
            full = x64.double() + torch.from_numpy(p64.reference).cuda().view(p64.batch, 2, 1, 1)
            diff = (x32.double() - x64).abs().amax(dim=(1, 2, 3))
            worst_w = max(worst_w, float((diff / full.abs().amax(dim=(1, 2, 3))).max()))
            worst_d = max(worst_d, float((diff / x64.abs().amax(dim=(1, 2, 3))).max()))
        if done % 500 == 0:
            print("step %4d: fp32 vs fp64 %.2e of max|W|, %.2e of max|dev|" % (done, worst_w, worst_d),
                  flush=True)
    # the two-step bound of the batch tests, 2e-6 of max|W| (the F tile is
    # rounded to FP32 where d sin^-2 A_theta W is ~1e6 times the state's
    # variation next to the poles, and the theta-mean mode does not damp it);
    # the kinetics are stable, so the error does not grow with the steps
    print("worst over %d steps: %.2e of max|W|, %.2e of max|dev|" % (big.steps, worst_w, worst_d))
    assert worst_w < 2e-6


def test_disk_256x512_400_step_gradient_vs_central_differences():
    """The gradient workload at its full length: FP32 forward, FP64 reverse
    sweep (the default), sqrt(T) checkpoints; against central differences
    (h = 1e-4, one Richardson step) of the FP64 device loss, along three
    seeded initial-state directions and in (d_u, d_v, a, b)."""
    from paper_2604_11558_amd.autograd import integrate
    w = workloads.WORKLOADS["disk_256x512"]
    grid = tg.Grid("disk", w.n)
    pert = workloads.perturbation(w)[None]
    p64 = tg.Plan(grid, w.diff, w.reaction, w.params, w.tau, "fp64")
    wref = p64.reference.copy()
    tgt = workloads.target_pattern(w) + wref[0, 0]
    tgt_t = torch.from_numpy(tgt).cuda()

    w0 = torch.from_numpy(pert).cuda().float().requires_grad_(True)
    diff = torch.tensor([w.diff], dtype=torch.float64, requires_grad=True)
    ab = torch.tensor([w.params], dtype=torch.float64, requires_grad=True)
    out = integrate(w0, grid, diff, ab, w.tau, w.steps, precision="fp32", w_ref=wref)
    loss = 0.5 * ((out[0, 0].double() + wref[0, 0] - tgt_t) ** 2).sum()
    loss.backward()
    g_w = w0.grad.double().cpu().numpy()
    g_p = np.concatenate([diff.grad.numpy()[0], ab.grad.numpy()[0]])

    def device_loss(p, d=w.diff, prm=w.params):
        plan = tg.Plan(grid, d, w.reaction, prm, w.tau, "fp64", w_ref=wref)
        x = plan.state_from_deviation(p)
        plan.run(x, w.steps)
        u = x[0, 0] + wref[0, 0]
        return 0.5 * float(((u - tgt_t) ** 2).sum())

    def rich(f, h=1e-4):
        c1 = (f(h) - f(-h)) / (2 * h)
        c2 = (f(h / 2) - f(-h / 2)) / h
        return (4 * c2 - c1) / 3

    L64 = device_loss(pert)
    # the FP32 forward moves u by up to 2e-7 of |u| ~ 1.1 per the parity
    # bound; relative to the residual u - target (~5e-4 here) the gradient
    # may move by that ratio: 2e-7 * 1.1 / 5e-4 = 4.4e-4
    rms = np.sqrt(2 * L64 / np.prod(w.n))
    tol = 2e-7 * 1.1 / rms
    print("loss: fp32 forward %.10e, fp64 %.10e; residual rms %.2e; tol %.1e" % (loss.item(), L64, rms, tol))
    rng = np.random.default_rng(26)
    for k in range(3):
        e = rng.standard_normal(pert.shape)
        fd = rich(lambda t: device_loss(pert + t * e))
        an = float(np.sum(g_w * e))
        print("direction %d: adjoint %.8e  central differences %.8e" % (k, an, fd), flush=True)
        assert abs(an - fd) < tol * abs(fd)
    fds = []
    for s in range(2):
        def f_d(t, s=s):
            d = list(w.diff)
            d[s] += t
            return device_loss(pert, d=d)
        fds.append(rich(f_d))
    for q in range(2):
        def f_p(t, q=q):
            prm = list(w.params)
            prm[q] += t
            return device_loss(pert, prm=prm)
        fds.append(rich(f_p))
    fds = np.array(fds)
    print("(d_u, d_v, a, b): adjoint", g_p, "central differences", fds)
    assert np.abs(g_p - fds).max() < tol * np.abs(fds).max()
