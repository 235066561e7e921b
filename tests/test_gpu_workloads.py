"""The benchmark-sized workloads against the FP64 oracle, at their full grid
sizes: the 32 x 64 disk (all 100 steps), the 64 x 64 x 128 ball in
lockstep with the oracle (error after every step), the 160 x 160
anomalous-diffusion disk, the 100^3 cylinder with three species in
split-bf16, and the gradient of the 256 x 512 disk."""
from types import SimpleNamespace

import numpy as np
import pytest

import paper_2604_11558_amd as tg
import workloads
from gpu_helpers import rel_err
from oracle import adjoint, assemble, reactions, splitee

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _setup(w, precision, n_steps_note=""):
    grid = tg.Grid(w.geometry, w.n, w.extent)
    plan = tg.Plan(grid, w.diff, w.reaction, w.params, w.tau, precision)
    pert = workloads.perturbation(w)
    eq = reactions.equilibrium(w.reaction, w.params)
    W = [eq[s] + assemble.from_layout(pert[s]) for s in range(w.n_species)]
    return plan, plan.state_from_deviation(pert[None]), W, eq


def _oracle_stepper(w, eq):
    se = splitee.make(w)
    react = lambda U: reactions.reaction(w.reaction, U, w.params)  # noqa: E731
    wd = eq if w.geometry in ("cylinder", "disk_lambda") else None
    return lambda W: se.step(W, react, w_dirichlet=wd)


def _full(plan, x):
    dev = x.double().cpu().numpy()[0]
    return dev + plan.reference[0].reshape((-1,) + (1,) * (dev.ndim - 1))


def test_disk_32x64_fp64_all_steps():
    w = workloads.WORKLOADS["disk_32x64"]
    plan, x, W, eq = _setup(w, "fp64")
    plan.run(x, w.steps)
    step = _oracle_stepper(w, eq)
    for _ in range(w.steps):
        W = step(W)
    ref = np.stack([assemble.to_layout(u) for u in W])
    err = rel_err(_full(plan, x), ref)
    print("disk 32x64 fp64, %d steps: %.2e" % (w.steps, err))
    assert err < 1e-12


def test_ball_64x64x128_lockstep_errors():
    """FP64 and FP32 against the oracle after each of 12 steps."""
    w = workloads.WORKLOADS["ball_64x64x128"]
    p64, x64, W, eq = _setup(w, "fp64")
    p32, x32, _, _ = _setup(w, "fp32")
    step = _oracle_stepper(w, eq)
    worst = {"fp64": 0.0, "fp32": 0.0}
    for it in range(12):
        p64.step(x64)
        p32.step(x32)
        W = step(W)
        ref = np.stack([assemble.to_layout(u) for u in W])
        e64, e32 = rel_err(_full(p64, x64), ref), rel_err(_full(p32, x32), ref)
        print("step %d: fp64 %.2e  fp32 %.2e" % (it + 1, e64, e32))
        worst["fp64"] = max(worst["fp64"], e64)
        worst["fp32"] = max(worst["fp32"], e32)
    assert worst["fp64"] < 1e-12 and worst["fp32"] < 2e-7, worst


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 2e-7)])
def test_disk_lambda_160x160(precision, tol):
    """The anomalous-diffusion disk (lambda = -1.95, alpha_1 = 500 kinetics)
    at full size, 200 steps; errors also relative to the deviation from the
    lifted equilibrium, which is what the steps change."""
    w = workloads.WORKLOADS["disk_lambda_160x160"]
    plan, x, W, eq = _setup(w, precision)
    steps = 200
    plan.run(x, steps)
    step = _oracle_stepper(w, eq)
    for _ in range(steps):
        W = step(W)
    ref = np.stack([assemble.to_layout(u) for u in W])
    got = _full(plan, x)
    err = rel_err(got, ref)
    dev = ref - np.asarray(eq).reshape(-1, 1, 1)
    dev_err = float(np.abs(got - ref).max() / np.abs(dev).max())
    print("disk_lambda 160x160 %s, %d steps: %.2e (deviation-relative %.2e)" % (precision, steps, err, dev_err))
    assert err < tol
    assert dev_err < (1e-8 if precision == "fp64" else 1e-3)


# split-bf16 on the cylinder (100 points per mode, d_w = 40): operand
# representation error 2^-17 (two terms) / 2^-25 (three terms) per product
# pair, three products per step
C3_TOL = {"bf16x2": 2e-6, "bf16x3": 5e-8}


@pytest.mark.parametrize("precision", ["bf16x2", "bf16x3"])
def test_cylinder_100cubed_split_bf16(precision):
    w = workloads.WORKLOADS["cylinder_100x100x100"]
    plan, x, W, eq = _setup(w, precision)
    assert plan.route == "fused"
    steps = 3
    plan.run(x, steps)
    step = _oracle_stepper(w, eq)
    for _ in range(steps):
        W = step(W)
    ref = np.stack([assemble.to_layout(u) for u in W])
    err = rel_err(_full(plan, x), ref)
    print("cylinder 100^3 %s, %d steps: %.2e" % (precision, steps, err))
    assert err < C3_TOL[precision]


def test_disk_256x512_gradient_fp32_forward():
    """FP32 forward with the checkpointed reverse sweep (FP64 adjoint plan),
    12 steps: the initial-state gradient along three seeded directions and
    the gradients in (d_u, d_v, a, b) against the oracle's discrete adjoint."""
    from paper_2604_11558_amd.autograd import integrate
    w = workloads.WORKLOADS["disk_256x512"]
    steps = 12
    grid = tg.Grid("disk", w.n)
    pert = workloads.perturbation(w)
    eq = reactions.equilibrium(w.reaction, w.params)
    plan = tg.Plan(grid, w.diff, w.reaction, w.params, w.tau, "fp32")
    target = eq[0] + assemble.from_layout(workloads.target_pattern(w))
    w0 = plan.state_from_deviation(pert[None]).requires_grad_(True)
    diff = torch.tensor([w.diff], dtype=torch.float64, requires_grad=True)
    ab = torch.tensor([w.params], dtype=torch.float64, requires_grad=True)
    out = integrate(w0, grid, diff, ab, w.tau, steps, precision="fp32", w_ref=plan.reference)
    u = out[0, 0].double() + float(plan.reference[0, 0])
    loss = 0.5 * ((u - torch.from_numpy(assemble.to_layout(target)).cuda()) ** 2).sum()
    loss.backward()
    W0 = [eq[s] + assemble.from_layout(pert[s]) for s in range(2)]
    wl = SimpleNamespace(geometry="disk", reaction=w.reaction, tau=w.tau, extent=w.extent, diff=w.diff,
                         params=w.params, n=w.n)
    L0, lam0, gd, gp = adjoint.loss_and_grad(wl, W0, target, steps)
    lam_ref = np.stack([assemble.to_layout(x) for x in lam0])
    g = w0.grad.double().cpu().numpy()[0]
    rng = np.random.default_rng(25)
    # the FP32 trajectory differs from the FP64 one by the forward parity
    # bound (2e-7 of |u| ~ 1, i.e. ~4e-4 of the residual u - target ~ 5e-4)
    tol = 2e-7 / 5e-4
    for k in range(3):
        e = rng.standard_normal(g.shape)
        a, b = float(np.sum(g * e)), float(np.sum(lam_ref * e))
        print("direction %d: %.6e vs %.6e" % (k, a, b))
        assert abs(a - b) < tol * abs(b)
    got = np.concatenate([diff.grad.numpy()[0], ab.grad.numpy()[0]])
    ref = np.concatenate([gd, gp])
    print("d, a, b gradients:", got, ref)
    assert np.abs(got - ref).max() < tol * np.abs(ref).max()
    assert abs(loss.item() - L0) < tol * L0
