"""GPU parity of the HIP path against the FP64 oracle (called through the
C interface).  FP64 must agree to 1e-12 relative; FP32 tolerances are
stated per test and derive from unit round-off 2^-24 times the chain
length and the conditioning of the eigenvector factors."""
import numpy as np
import pytest

from gpu_helpers import Case, rel_err
from oracle import assemble, reactions

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# small grids spanning several 64-wide tiles plus ragged tails, and minimal sizes
GRIDS = [
    ("disk", (37, 70)), ("disk", (3, 3)),
    ("sphere", (70, 45)), ("sphere", (3, 4)),
    ("ball", (20, 24, 37)), ("ball", (3, 3, 3)),
    ("cylinder", (27, 30, 19)), ("cylinder", (3, 4, 3)),
    ("disk_lambda", (37, 70)), ("disk_lambda", (3, 3)),
]
TOL = {"fp64": 1e-12, "fp32": 2e-6}


def _hooks(case, precision):
    plan = case.plan
    x = case.device_state()
    out = torch.empty_like(x)
    return plan, x, out


@pytest.mark.parametrize("geometry,n", GRIDS)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_diffusion_operator(geometry, n, precision):
    case = Case(geometry, n, precision, seed=1, amplitude=1.0)
    plan, x, out = _hooks(case, precision)
    plan.apply_operator(x, out, "diffusion")
    got = out.double().cpu().numpy()[0]
    for s in range(case.ns):
        P = case.to_species(case.pert[0])[s]
        ref = assemble.to_layout(case.oracles[0].apply_M(P, s))
        err = rel_err(got[s], ref)
        assert err < (1e-13 if precision == "fp64" else 1e-6), err


@pytest.mark.parametrize("geometry,n", GRIDS[:3] + [("cylinder", (27, 30, 19)), ("disk_lambda", (37, 70))])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_reaction(geometry, n, precision):
    ns = 3 if geometry == "cylinder" else 2
    case = Case(geometry, n, precision, seed=2, n_species=ns, amplitude=0.3)
    plan, x, out = _hooks(case, precision)
    plan.apply_operator(x, out, "reaction")
    got = out.double().cpu().numpy()[0]
    W = case.oracle_full(0)
    G = reactions.reaction(case.kind, W, tuple(case.params[0]))
    for s in range(ns):
        ref = assemble.to_layout(G[s])
        err = float(np.abs(got[s] - ref).max() / max(1.0, np.abs(ref).max()))
        # fp32: input and output each rounded once (2 x 2^-24 relative)
        assert err < (1e-15 if precision == "fp64" else 3e-7), err


@pytest.mark.parametrize("geometry,n", GRIDS)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("tau", [5e-3, 0.3])
@pytest.mark.parametrize("route", ["fused", "generic"])
def test_split_phi1(geometry, n, precision, tau, route):
    case = Case(geometry, n, precision, tau=tau, seed=3, amplitude=1.0)
    case.plan.set_route(route)
    plan, x, out = _hooks(case, precision)
    plan.split_phi1(x, out)
    got = out.double().cpu().numpy()[0]
    for s in range(case.ns):
        F = case.to_species(case.pert[0])[s]
        ref = assemble.to_layout(case.oracles[0].split_phi1(F, s))
        err = rel_err(got[s], ref)
        assert err < TOL[precision], (s, err)


@pytest.mark.parametrize("geometry,n", GRIDS)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("route", ["fused", "generic", "fused_stencil_apart"])
def test_steps(geometry, n, precision, route):
    ns = 3 if geometry == "cylinder" else 2
    case = Case(geometry, n, precision, tau=5e-3, seed=4, n_species=ns)
    case.plan.set_route(route)
    assert case.plan.route == route
    x = case.device_state()
    case.plan.run(x, 10)
    got = case.full_from_device(x)
    ref = case.oracle_run(10)
    err = rel_err(got, ref)
    assert err < (1e-12 if precision == "fp64" else 2e-7), err
    # relative to the deviation from equilibrium too (FP64 only; FP32 is checked against the full state)
    dev_ref = ref - case.plan.reference.reshape(ref.shape[:2] + (1,) * (ref.ndim - 2))
    dev_err = np.abs(got - ref).max() / np.abs(dev_ref).max()
    assert dev_err < (1e-9 if precision == "fp64" else 1e-3), dev_err


def test_batch_with_per_instance_parameters():
    params = [(0.1, 0.9), (0.15, 0.8), (0.06, 1.05)]
    diff = [(1.0, 20.0), (1.0, 12.0), (1.0, 35.0)]
    case = Case("sphere", (40, 33), "fp64", tau=1e-2, seed=5, batch=3, params=params, diff=diff)
    x = case.device_state()
    case.plan.run(x, 6)
    assert rel_err(case.full_from_device(x), case.oracle_run(6)) < 1e-12


def test_full_size_ball_fp64_and_fp32():
    """The 64 x 64 x 128 ball with the benchmark's launch configuration
    (fused route: two launches per step), all elements after 3 steps."""
    n = (64, 64, 128)
    ref = None
    for prec, tol in (("fp64", 1e-12), ("fp32", 2e-7)):
        case = Case("ball", n, prec, tau=5e-3, seed=3)
        assert case.plan.route == "fused" and len(case.plan.chain()) == 2
        if ref is None:
            ref = case.oracle_run(3)
        x = case.device_state()
        case.plan.run(x, 3)
        err = rel_err(case.full_from_device(x), ref)
        assert err < tol, (prec, err)


def test_equilibrium_is_stationary():
    case = Case("cylinder", (12, 10, 9), "fp64", n_species=3, amplitude=0.0)
    x = case.device_state()
    case.plan.run(x, 5)
    assert float(x.abs().max()) < 1e-14


# split-bf16 precisions: operand representation error 2^-17 per term pair
# (two terms) or 2^-25 (three terms), times the chain length and the
# eigenvector conditioning; bounds below hold with a margin of about 5x
# over the measured errors.
BF16_TOL = {"bf16x2": {"split": 6e-5, "steps": 1.5e-6}, "bf16x3": {"split": 3.5e-6, "steps": 3e-8}}
BF16_GRIDS = [("disk", (37, 70)), ("sphere", (70, 45)), ("ball", (20, 24, 37)),
              ("cylinder", (27, 30, 19)), ("ball", (64, 64, 128)), ("disk_lambda", (37, 70))]


@pytest.mark.parametrize("geometry,n", BF16_GRIDS)
@pytest.mark.parametrize("precision", ["bf16x2", "bf16x3"])
def test_bf16_split_phi1(geometry, n, precision):
    case = Case(geometry, n, precision, tau=5e-3, seed=3, amplitude=1.0)
    assert case.plan.route == "fused"
    plan, x, out = _hooks(case, precision)
    plan.split_phi1(x, out)
    got = out.double().cpu().numpy()[0]
    errs = []
    for s in range(case.ns):
        F = case.to_species(case.pert[0])[s]
        ref = assemble.to_layout(case.oracles[0].split_phi1(F, s))
        errs.append(rel_err(got[s], ref))
    print(geometry, n, precision, "split errors", errs)
    assert max(errs) < BF16_TOL[precision]["split"], errs


@pytest.mark.parametrize("geometry,n", BF16_GRIDS[:4])
@pytest.mark.parametrize("precision", ["bf16x2", "bf16x3"])
@pytest.mark.parametrize("route", ["fused", "fused_stencil_apart"])
def test_bf16_steps(geometry, n, precision, route):
    ns = 3 if geometry == "cylinder" else 2
    case = Case(geometry, n, precision, tau=5e-3, seed=4, n_species=ns)
    case.plan.set_route(route)
    x = case.device_state()
    case.plan.run(x, 10)
    err = rel_err(case.full_from_device(x), case.oracle_run(10))
    print(geometry, n, precision, route, "10-step error", err)
    assert err < BF16_TOL[precision]["steps"], err


def test_bf16_rejects_generic_route():
    import paper_2604_11558_amd as tg
    case = Case("disk", (12, 16), "bf16x3")
    with pytest.raises(tg.TGError):
        case.plan.set_route("generic")


# per-slice route (ball phi mode, cylinder theta mode by per-radius dense factors)
PER_SLICE_GRIDS = [("ball", (20, 24, 37)), ("ball", (3, 3, 3)), ("cylinder", (27, 30, 19)), ("cylinder", (3, 4, 3))]


@pytest.mark.parametrize("geometry,n", PER_SLICE_GRIDS)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_per_slice_route_steps(geometry, n, precision):
    ns = 3 if geometry == "cylinder" else 2
    case = Case(geometry, n, precision, tau=5e-3, seed=4, n_species=ns)
    case.plan.set_route("per_slice")
    assert case.plan.route == "per_slice"
    x = case.device_state()
    case.plan.run(x, 10)
    err = rel_err(case.full_from_device(x), case.oracle_run(10))
    print(geometry, n, precision, "per-slice 10-step error", err)
    assert err < (1e-12 if precision == "fp64" else 2e-7), err


@pytest.mark.parametrize("geometry,n", PER_SLICE_GRIDS[::2])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 2e-6)])
def test_per_slice_split_hook(geometry, n, precision, tol):
    ns = 3 if geometry == "cylinder" else 2
    case = Case(geometry, n, precision, tau=0.3, seed=5, n_species=ns, amplitude=1.0)
    case.plan.set_route("per_slice")
    plan, x, out = _hooks(case, precision)
    plan.split_phi1(x, out)
    got = out.double().cpu().numpy()[0]
    for s in range(ns):
        F = case.to_species(case.pert[0])[s]
        ref = assemble.to_layout(case.oracles[0].split_phi1(F, s))
        assert rel_err(got[s], ref) < tol


def test_per_slice_batch_with_per_instance_diffusion():
    diff = [(1.0, 20.0), (1.0, 7.0)]
    case = Case("ball", (12, 10, 14), "fp64", tau=1e-2, seed=6, batch=2, diff=diff)
    case.plan.set_route("per_slice")
    x = case.device_state()
    case.plan.run(x, 5)
    assert rel_err(case.full_from_device(x), case.oracle_run(5)) < 1e-12


def test_per_slice_full_size_ball_fp32():
    case = Case("ball", (64, 64, 128), "fp32", tau=5e-3, seed=3)
    case.plan.set_route("per_slice")
    x = case.device_state()
    case.plan.run(x, 3)
    assert rel_err(case.full_from_device(x), case.oracle_run(3)) < 2e-7


def test_per_slice_route_is_refused_elsewhere():
    import paper_2604_11558_amd as tg
    for geometry, n, prec in (("disk", (8, 12), "fp64"), ("sphere", (12, 9), "fp32"), ("ball", (6, 8, 7), "bf16x3")):
        case = Case(geometry, n, prec)
        with pytest.raises(tg.TGError):
            case.plan.set_route("per_slice")
