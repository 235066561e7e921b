"""Throughput of the split exponential Euler step on one MI355X.

Workload (default): the 64 x 64 x 128 ball (n_rho, n_theta, n_phi), two
Schnakenberg species (d = 1, 20; a = 0.1, b = 0.9), tau = 5e-3, initial data
equilibrium + 1e-3 U(0,1) (seed 3), synthetic.  One "step" is one full step
of the method on the whole state (stencil + reaction, the five mu-mode
products of eq. (ee_ball) and the update).  The headline value is the FP32
MFMA path in dof-steps/s (dof = points x species); the FP64 path is timed
beside it, and the FP32 result is compared with FP64 after the same steps.

Prints one JSON line.  Only the cpu_baseline leg calls the oracle.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

METRIC = "dof-steps/s per GPU (FP32-MFMA vs FP64) at stated rel. error vs FP64 oracle"
PEAK = {"fp64": 78.6e12, "fp32": 157.3e12}  # dense MFMA FLOP/s, MI355X
HBM_PEAK = 8.0e12


def cpu_model() -> str:
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def blas_threads() -> int:
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        return max([i.get("num_threads", 1) for i in info] + [1])
    except Exception:
        return os.cpu_count() or 1


def time_gpu_run(plan, x, steps, warmup, torch):
    """Wall-clock per step with synchronisation on both sides (graph replay)."""
    if warmup:
        plan.run(x, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.run(x, steps)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def time_chain_op(plan, op, x, y, reps, torch):
    """Average duration of one chain product, HIP events on its stream."""
    stream = torch.cuda.current_stream()
    for _ in range(5):
        plan.apply_chain_op(op, x, y, stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        plan.apply_chain_op(op, x, y, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / reps


def cpu_baseline(w, pert, steps):
    """Oracle steps on the host (set-up and one warm-up step excluded)."""
    from oracle import reactions, splitee
    se = splitee.make(w)
    Ws = splitee.initial_state(w, pert)
    react = lambda U: reactions.reaction(w.reaction, U, w.params)  # noqa: E731
    wd = reactions.equilibrium(w.reaction, w.params) if w.geometry == "cylinder" else None
    Ws = se.step(Ws, react, w_dirichlet=wd)
    t0 = time.perf_counter()
    for _ in range(steps):
        Ws = se.step(Ws, react, w_dirichlet=wd)
    per_step = (time.perf_counter() - t0) / steps
    return w.dof / per_step, per_step, splitee.stack_layout(Ws)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=16)
    ap.add_argument("--workload", default="ball_64x64x128")
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); "
              "multi-GPU sharding is not part of this build", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2604_11558_amd as tg

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    w = workloads.WORKLOADS[args.workload]
    pert = workloads.perturbation(w)
    grid = tg.Grid(w.geometry, w.n, w.extent)

    res = {}
    states = {}
    for prec in ("fp64", "fp32"):
        t0 = time.perf_counter()
        plan = tg.Plan(grid, w.diff, w.reaction, w.params, w.tau, prec)
        setup = time.perf_counter() - t0
        x = plan.state_from_deviation(pert)
        xw = plan.state_from_deviation(pert)
        plan.run(xw, args.warmup)  # warm-up on a separate state (graph capture, clocks)
        torch.cuda.synchronize()
        sec = time_gpu_run(plan, x, args.steps, 0, torch)
        states[prec] = x.double().cpu().numpy()
        # per-launch timing of the step's kernels (HIP events on the launch stream)
        chain = plan.chain()
        bufs = [x, torch.empty_like(x), torch.empty_like(x)]
        op_times = []
        for i in range(len(chain)):
            src = bufs[0] if i == 0 else bufs[1 + (i - 1) % 2]
            dst = bufs[1 + i % 2]
            op_times.append(time_chain_op(plan, i, src, dst, 200, torch))
        dom = int(np.argmax(op_times))
        route = plan.route
        # the other routes for comparison
        other = {}
        for rname in ("generic", "fused_stencil_apart"):
            plan.set_route(rname)
            xg = plan.state_from_deviation(pert)
            plan.run(xg, args.warmup)
            other[rname] = time_gpu_run(plan, xg, min(args.steps, 200), 0, torch)
            del xg
        plan.set_route(route)
        res[prec] = dict(sec=sec, setup=setup, op_times=op_times, dom=dom,
                         flops=[f for _, f in chain], modes=[m for m, _ in chain],
                         ref=plan.reference.copy(), route=route, other=other)
        del plan, x, xw, bufs
        torch.cuda.empty_cache()

    # split-bf16 precisions of the same step (fused route)
    bf = {}
    for prec in ("bf16x3", "bf16x2"):
        plan = tg.Plan(grid, w.diff, w.reaction, w.params, w.tau, prec)
        xw = plan.state_from_deviation(pert)
        plan.run(xw, args.warmup)
        x = plan.state_from_deviation(pert)
        sec = time_gpu_run(plan, x, args.steps, 0, torch)
        full = x.double().cpu().numpy() + plan.reference[:, :, None, None, None]
        bf[prec] = dict(sec=sec, full=full)
        del plan, x, xw
        torch.cuda.empty_cache()

    dof = w.dof
    v32 = dof / res["fp32"]["sec"]
    v64 = dof / res["fp64"]["sec"]
    ref64 = states["fp64"] + res["fp64"]["ref"][:, :, None, None, None]
    full32 = states["fp32"] + res["fp32"]["ref"][:, :, None, None, None]
    err_32_64 = float(np.abs(full32 - ref64).max() / np.abs(ref64).max())
    dev64 = states["fp64"]
    err_32_64_dev = float(np.abs(full32 - ref64).max() / max(np.abs(dev64).max(), 1e-300))

    r = res["fp32"]
    dom = r["dom"]
    achieved = r["flops"][dom] / r["op_times"][dom]
    out = {
        "metric": METRIC,
        "value": v32,
        "unit": "dof-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["fp32"]["sec"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "geometry": w.geometry, "n": list(w.n),
                   "species": w.n_species, "dof": dof, "tau": w.tau,
                   "reaction": w.reaction, "seed": w.seed},
        "fp64": {"value": v64, "ms_per_step": res["fp64"]["sec"] * 1e3, "dtype": "f64"},
        "speedup_fp32_vs_fp64": v32 / v64,
        "split_bf16": {p: {"value": dof / bf[p]["sec"], "ms_per_step": bf[p]["sec"] * 1e3,
                           "rel_err_vs_fp64_after_steps": float(np.abs(bf[p]["full"] - ref64).max()
                                                                / np.abs(ref64).max())}
                       for p in bf},
        "rel_err_fp32_vs_fp64": {"after_steps": args.steps, "vs_max_state": err_32_64,
                                 "vs_max_deviation": err_32_64_dev},
        "route": res["fp32"]["route"],
        "launch_us": {p: [t * 1e6 for t in res[p]["op_times"]] for p in res},
        "ms_per_step_other_routes": {p: {k: v * 1e3 for k, v in res[p]["other"].items()} for p in res},
        "plan_setup_s": {p: res[p]["setup"] for p in res},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK["fp32"] / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK["fp32"], "traffic": None,
                     "kernel": f"launch {dom} of the {r['route']} route (leading mode {r['modes'][dom]})",
                     "flops_per_launch": r["flops"][dom],
                     "avg_launch_us": r["op_times"][dom] * 1e6},
    }
    # step-level roofline (whole chain's flops in one step vs MFMA peak)
    step_flops = sum(r["flops"])
    out["step_roofline"] = {"flops_per_step": step_flops,
                            "fp32_frac": step_flops / res["fp32"]["sec"] / PEAK["fp32"],
                            "fp64_frac": step_flops / res["fp64"]["sec"] / PEAK["fp64"]}

    if not args.no_cpu:
        v_cpu, per_step, ws = cpu_baseline(w, pert, args.cpu_steps)
        out["cpu_baseline"] = {"value": v_cpu, "unit": "dof-steps/s", "cores": blas_threads(),
                               "kind": "oracle", "host_cpu": cpu_model(),
                               "sample": f"{args.cpu_steps} steps of {w.name} (FP64 NumPy/SciPy "
                                         f"oracle), s/step = {per_step:.3f}"}
        # FP32 GPU path against the oracle on the same sample
        g32 = tg.Plan(grid, w.diff, w.reaction, w.params, w.tau, "fp32")
        x = g32.state_from_deviation(pert)
        g32.run(x, args.cpu_steps + 1)
        got = x.double().cpu().numpy() + g32.reference[:, :, None, None, None]
        out["rel_err_fp32_vs_oracle"] = {"after_steps": args.cpu_steps + 1,
                                         "vs_max_state": float(np.abs(got[0] - ws).max() / np.abs(ws).max())}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
