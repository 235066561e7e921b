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
PEAK = {"fp64": 78.6e12, "fp32": 157.3e12, "bf16": 2.5e15}  # dense MFMA FLOP/s, MI355X
HBM_PEAK = 8.0e12
KERNEL_SOURCES = ("fused.hip", "fused.hpp", "stencil_dev.hpp", "kernels.hpp", "phi_dev.hpp")
COPY_BYTES = 256 << 20
# HBM traffic per launch (FETCH_SIZE + WRITE_SIZE per dispatch, scaled by
# the copy calibration), keyed "route:launch:tiles", from the rocprofv3
# counter runs of `bench.py --profile` summarised under profiles/; valid
# only while the kernel sources hash to TRAFFIC_DIGEST.
TRAFFIC = {"fused:0:16,64": 11036238, "fused:1:16,64": 13325577,
           "fused_stencil_apart:0:32,64": 9694866, "fused_stencil_apart:1:32,64": 13325586,
           "fused_stencil_apart:0:16,64": 9651842, "fused_stencil_apart:1:16,64": 13325574}
TRAFFIC_DIGEST = "2e1a43c1dd00faa5e5ddd2e2323620ec0eb78627215e8ea681dc173f1db28a13"


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


CAPTURE_S = {}


def time_gpu_run(plan, x, steps, warmup, torch, label=None):
    """Wall-clock per step with synchronisation on both sides (graph replay).

    The graphs tg_run replays are captured and instantiated before the
    warm-up (tg_run_prepare), so the timed steps are steady state whatever
    ``warmup`` is; the capture time is kept in CAPTURE_S[label]."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.prepare_run(x)
    if label:
        CAPTURE_S[label] = time.perf_counter() - t0
    if warmup:
        plan.run(x, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.run(x, steps)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def time_chain_op(plan, op, x, y, reps, torch):
    """Average duration of one launch of the step, repeated back to back
    between two HIP events on its stream."""
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


def cpu_baseline(w, pert, budget_s):
    """Oracle steps on the host for about ``budget_s`` seconds (set-up and
    one warm-up step excluded; at least 3 steps)."""
    from oracle import reactions, splitee
    se = splitee.make(w)
    Ws = splitee.initial_state(w, pert)
    react = lambda U: reactions.reaction(w.reaction, U, w.params)  # noqa: E731
    wd = reactions.equilibrium(w.reaction, w.params) if w.geometry == "cylinder" else None
    Ws = se.step(Ws, react, w_dirichlet=wd)
    n = 0
    t0 = time.perf_counter()
    while n < 3 or time.perf_counter() - t0 < budget_s:
        Ws = se.step(Ws, react, w_dirichlet=wd)
        n += 1
    per_step = (time.perf_counter() - t0) / n
    return w.dof / per_step, per_step, n, splitee.stack_layout(Ws)


def step_roofline(flops, sec, peak, what, nbytes=None):
    """Fraction of the MFMA peak (and of HBM, given the algorithmic bytes)
    that one step's algorithmic work reaches in ``sec`` seconds."""
    r = {"what": what, "flops": flops, "achieved_tflops": flops / sec / 1e12, "peak_tflops": peak / 1e12,
         "frac": flops / sec / peak}
    if nbytes is not None:
        r.update({"bytes": nbytes, "achieved_gbs": nbytes / sec / 1e9, "hbm_frac": nbytes / sec / HBM_PEAK})
    return r


def kernel_sources_digest() -> str:
    """SHA-256 of the HIP sources the fused launches are built from."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2604_11558_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def other_workloads(tg, torch, steps):
    """Throughput of the other benchmark-shaped workloads (context lines)."""
    out = {}
    # 64 x (256 x 512) + 32 x (128 x 256) sphere instances, FP32, grouped launches
    big, small = workloads.WORKLOADS["sphere_256x512"], workloads.WORKLOADS["sphere_128x256"]
    prm = workloads.sphere_batch_params(big.batch + small.batch)
    plans, states = [], []
    for wl, rows in ((big, prm[:big.batch]), (small, prm[big.batch:])):
        diff = np.stack([np.ones(wl.batch), rows[:, 2]], axis=1)
        plan = tg.Plan(tg.Grid("sphere", wl.n), diff, "schnakenberg", rows[:, :2], wl.tau, "fp32", wl.batch)
        plans.append(plan)
        states.append(plan.state_from_deviation(workloads.batch_perturbations(wl)))
    tg.group_autotune(plans, states, iters=5)
    info = tg.group_info(plans, states)
    tg.group_run(plans, states, 16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tg.group_run(plans, states, steps)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    dof = big.dof + small.dof
    flops = sum(f for p in plans for _, f in p.chain())  # per step, both grids
    out["sphere_64x256x512_32x128x256_fp32_grouped"] = {
        "value": dof / sec, "unit": "dof-steps/s", "ms_per_step": sec * 1e3, "dof": dof,
        "launches_per_step": info["launches_per_step"], "grouped": info["grouped"], "route": plans[0].route,
        "tiles": [p.tiles() for p in plans],
        "roofline": step_roofline(flops, sec, PEAK["fp32"], "step: every grouped launch of one step")}
    del plans, states
    torch.cuda.empty_cache()
    # 100^3 cylinder, 3 species: split-bf16 (the configured precision) with
    # FP32 and plain FP64 beside it, each after the same W + K steps; the
    # reduced precisions' deviation from FP64 against the scheme's own
    # time-discretisation error (step doubling in FP64)
    wl = workloads.WORKLOADS["cylinder_100x100x100"]
    grid = tg.Grid(wl.geometry, wl.n, wl.extent)
    pert = workloads.perturbation(wl)[None]
    cyl, full = {}, {}
    for prec in ("fp64", "fp32", "bf16x2", "bf16x3"):
        plan = tg.Plan(grid, wl.diff, wl.reaction, wl.params, wl.tau, prec)
        x = plan.state_from_deviation(pert)
        plan.autotune(x, iters=10)
        x = plan.state_from_deviation(pert)
        sec = time_gpu_run(plan, x, steps, 16, torch)
        full[prec] = x.double().cpu().numpy() + plan.reference[:, :, None, None, None]
        chain = plan.chain()
        bufs = [plan.state_from_deviation(pert), torch.empty_like(x), torch.empty_like(x)]
        op_t = [time_chain_op(plan, i, bufs[0] if i == 0 else bufs[1 + (i - 1) % 2], bufs[1 + i % 2], 50, torch)
                for i in range(len(chain))]
        del bufs
        dom = int(np.argmax(op_t))
        terms = {"bf16x2": 3, "bf16x3": 6}.get(prec, 1)  # MFMA products per algorithmic product
        peak = {"fp64": PEAK["fp64"], "fp32": PEAK["fp32"]}.get(prec, PEAK["bf16"])
        ebytes = 8 if prec == "fp64" else 4
        # one read of the launch's input and one write of its output (the
        # update launch also reads the state)
        nbytes = wl.dof * ebytes * (3 if dom == len(chain) - 1 else 2)
        cyl[prec] = {"value": wl.dof / sec, "unit": "dof-steps/s", "ms_per_step": sec * 1e3, "dof": wl.dof,
                     "route": plan.route, "tiles": plan.tiles(), "launch_us": [t * 1e6 for t in op_t],
                     "roofline": {
                         "kernel": f"launch {dom} (leading mode {chain[dom][0]})",
                         "mfma": {"achieved": terms * chain[dom][1] / op_t[dom] / 1e12, "peak": peak / 1e12,
                                  "unit": "TFLOP/s", "frac": terms * chain[dom][1] / op_t[dom] / peak,
                                  "flops_per_launch": terms * chain[dom][1]},
                         "hbm": {"achieved": nbytes / op_t[dom] / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                                 "frac": nbytes / op_t[dom] / HBM_PEAK, "algorithmic_bytes_per_launch": nbytes},
                         "avg_launch_us": op_t[dom] * 1e6},
                     "step_roofline": step_roofline(terms * sum(f for _, f in chain), sec, peak,
                                                    "step: every launch", 2 * wl.dof * ebytes)}
        del plan, x
        torch.cuda.empty_cache()
    half = tg.Plan(grid, wl.diff, wl.reaction, wl.params, wl.tau / 2, "fp64")
    xh = half.state_from_deviation(pert)
    half.run(xh, 2 * (steps + 16))
    ref = full["fp64"]
    dev = np.abs(ref - half.reference[:, :, None, None, None]).max()
    t_err = 2.0 * float(np.abs(ref - (xh.double().cpu().numpy() + half.reference[:, :, None, None, None])).max()
                        / np.abs(ref).max())
    del half, xh
    for prec in ("fp32", "bf16x2", "bf16x3"):
        e = float(np.abs(full[prec] - ref).max())
        cyl[prec]["rel_err_vs_fp64"] = {"after_steps": steps + 16, "vs_max_state": e / np.abs(ref).max(),
                                        "vs_max_deviation": e / dev}
        cyl[prec]["equal_accuracy"] = bool(e / np.abs(ref).max() < t_err)
        cyl[prec]["speedup_vs_fp64"] = cyl[prec]["value"] / cyl["fp64"]["value"]
    for prec in cyl:
        out[f"cylinder_100x100x100_{prec}"] = cyl[prec]
    out["cylinder_100x100x100_time_discretisation_error"] = {
        "after_steps": steps + 16, "vs_max_state": t_err, "method": "2 |W_tau - W_tau/2| / |W| (FP64)"}
    # steady-state indicators on the 64 x 64 x 128 ball, FP32 (fused into the
    # update launch plus one small summing launch per recorded step)
    wl = workloads.WORKLOADS["ball_64x64x128"]
    grid = tg.Grid(wl.geometry, wl.n, wl.extent)
    plan = tg.Plan(grid, wl.diff, wl.reaction, wl.params, wl.tau, "fp32")
    x = plan.state_from_deviation(workloads.perturbation(wl)[None])
    plan.autotune(x, iters=10)
    plain = time_gpu_run(plan, x, steps, 16, torch)
    res = {"plain_ms_per_step": plain * 1e3}
    for every in (1, 10):
        plan.run_diag(x, 2 * every, every)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rec = plan.run_diag(x, steps, every)
        torch.cuda.synchronize()
        res[f"every_{every}_ms_per_step"] = (time.perf_counter() - t0) * 1e3 / steps
        res[f"every_{every}_last_record"] = rec[-1, 0].cpu().numpy().tolist()
    out["ball_64x64x128_fp32_indicators"] = res
    del plan, x
    # bulk-surface ball (30 x 50 x 30) + sphere (50 x 30), Section 5.5's grid
    bs = workloads.BULK_SURFACE
    nb = bs["n"]
    cpl = (55.0, 5.0 / 12.0, 5.0 / 12.0, 5.0, 5.0)  # zeta1, zeta2, zeta3, eta1, eta2
    db, dsf = workloads.bulk_surface_perturbations(nb, bs["seed"], bs["amplitude"])
    for prec in ("fp64", "fp32"):
        bulk = tg.Plan(tg.Grid("ball", nb), [(1.0, 10.0)], "schnakenberg_scaled", (0.1, 0.9, 55.0),
                       bs["tau"], prec)
        surf = tg.Plan(tg.Grid("sphere", nb[1:]), [(1.0, 10.0)], "schnakenberg_scaled", (0.1, 0.9, 55.0),
                       bs["tau"], prec)
        xb = bulk.state_from_deviation(db[None])
        xs = surf.state_from_deviation(dsf[None])
        tg.coupled_run(bulk, surf, xb, xs, cpl, 16)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tg.coupled_run(bulk, surf, xb, xs, cpl, steps)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        dof = 2 * int(np.prod(nb)) + 2 * nb[1] * nb[2]
        out[f"ball_sphere_30x50x30_coupled_{prec}"] = {
            "value": dof / sec, "unit": "dof-steps/s", "ms_per_step": sec * 1e3, "dof": dof,
            "paper_run_seconds_at_this_rate": bs["steps"] * sec}
        del bulk, surf, xb, xs
    # bulk-surface DIB system, cylinder 140 x 140 x 25 + bottom disk 140 x 140
    # (Section 5.6): linear bulk kinetics (alpha1, alpha2, beta1, beta2) =
    # (1, 1, 1, 1), delta = 1; DIB surface kinetics with zeta = (1, 10, 1,
    # 30, 0.5), eta = (3, 2.5, 0.2, eta4, 1.5), epsilon = 20, and the
    # coupling (alpha3, beta3) = (0.1, 0.1); eta4 is the value the paper
    # prints as a formula, which makes (u, v, r, s) = (1, 1, 0, 0.5) an
    # equilibrium
    bc = workloads.BULK_SURFACE_CYLINDER
    nc = bc["n"]
    eta4 = 1.0 * 3.0 * (1.0 - 0.5) * (1.0 - 0.2 + 0.2 * 0.5) / (0.5 * (1.0 + 0.2 * 0.5))
    dib = (1.0, 10.0, 1.0, 30.0, 0.5, 3.0, 2.5, 0.2, eta4, 1.5)
    dbc, dsc = workloads.bulk_surface_cylinder_perturbations(nc, bc["seed"], bc["amplitude"])
    for prec in ("fp64", "fp32"):
        bulk = tg.Plan(tg.Grid("cylinder", nc, bc["extent"]), [(1.0, 1.0)], "linear", (1.0, 1.0, 1.0, 1.0),
                       bc["tau"], prec)
        surf = tg.Plan(tg.Grid("disk", nc[:2], (bc["extent"][0], 1.0)), [(1.0, 20.0)], "dib", dib, bc["tau"], prec)
        xb = bulk.state_from_deviation(dbc[None])
        xs = surf.state_from_deviation(dsc[None])
        tg.coupled_run(bulk, surf, xb, xs, (0.1, 0.1), 16)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tg.coupled_run(bulk, surf, xb, xs, (0.1, 0.1), steps)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        dof = 2 * int(np.prod(nc)) + 2 * nc[0] * nc[1]
        out[f"cylinder_disk_140x140x25_coupled_{prec}"] = {
            "value": dof / sec, "unit": "dof-steps/s", "ms_per_step": sec * 1e3, "dof": dof,
            "routes": [bulk.route, surf.route], "paper_run_seconds_at_this_rate": bc["steps"] * sec}
        del bulk, surf, xb, xs
    # 32 x 64 disk, 100 steps of 1e-2 (a latency-bound 4096-dof problem):
    # autotuned, which picks the resident route (every step of a run in one
    # launch, one workgroup holding the states in LDS) over the fused one
    # (a stencil launch and a fused launch per step, graph-replayed); then
    # the fused route for comparison, and a batch of 256 instances with
    # their own parameters on the resident route (one workgroup each)
    wl = workloads.WORKLOADS["disk_32x64"]
    grid = tg.Grid(wl.geometry, wl.n, wl.extent)
    nrun = max(steps, wl.steps)
    for prec in ("fp64", "fp32"):
        plan = tg.Plan(grid, wl.diff, wl.reaction, wl.params, wl.tau, prec)
        x = plan.state_from_deviation(workloads.perturbation(wl)[None])
        plan.autotune(x, iters=100)
        plan.run(x, 16)
        sec = time_gpu_run(plan, x, nrun, 0, torch)
        route = plan.route
        flops = sum(f for _, f in plan.chain())  # per step: (2 n_rho + 4 n_theta) per dof
        peak = 78.6 if prec == "fp64" else 157.3
        plan.set_route("fused")
        plan.run(x, 16)
        sec_fused = time_gpu_run(plan, x, nrun, 0, torch)
        out[f"disk_32x64_{prec}"] = {"value": wl.dof / sec, "unit": "dof-steps/s", "ms_per_step": sec * 1e3,
                                     "steps_per_s": 1.0 / sec, "dof": wl.dof, "route": route,
                                     "steps_timed": nrun,
                                     "mfma_tflops": flops / sec / 1e12,
                                     "frac_of_one_cu_mfma_peak": flops / sec / 1e12 / (peak / 256),
                                     "fused_route": {"ms_per_step": sec_fused * 1e3,
                                                     "launches_per_step": len(plan.run_timed(x.clone(), 1))}}
        del plan, x
        B = 256
        prm = workloads.sphere_batch_params(B)  # (a, b, d2) uniform in the sphere batch's ranges
        plan = tg.Plan(grid, np.stack([np.ones(B), prm[:, 2]], axis=1), wl.reaction, prm[:, :2], wl.tau, prec, B)
        x = plan.state_from_deviation(np.repeat(workloads.perturbation(wl)[None], B, axis=0))
        plan.set_route("resident")
        plan.run(x, 16)
        sec = time_gpu_run(plan, x, nrun, 0, torch)
        out[f"disk_32x64_batch256_resident_{prec}"] = {"value": B * wl.dof / sec, "unit": "dof-steps/s",
                                                       "ms_per_step": sec * 1e3, "instances": B,
                                                       "mfma_tflops": B * flops / sec / 1e12,
                                                       "frac_of_mfma_peak": B * flops / sec / 1e12 / peak}
        del plan, x
    # 160 x 160 anomalous-diffusion disk (lambda = -1.95), FP64 and FP32
    wl = workloads.WORKLOADS["disk_lambda_160x160"]
    grid = tg.Grid(wl.geometry, wl.n, wl.extent)
    for prec in ("fp64", "fp32"):
        plan = tg.Plan(grid, wl.diff, wl.reaction, wl.params, wl.tau, prec)
        x = plan.state_from_deviation(workloads.perturbation(wl)[None])
        plan.autotune(x, iters=10)
        plan.run(x, 16)
        sec = time_gpu_run(plan, x, steps, 0, torch)
        out[f"disk_lambda_160x160_{prec}"] = {"value": wl.dof / sec, "unit": "dof-steps/s",
                                              "ms_per_step": sec * 1e3, "dof": wl.dof,
                                              "route": plan.route}
        del plan, x
    # 256 x 512 disk: FP32 forward + checkpointed reverse sweep, 400 steps
    from paper_2604_11558_amd.autograd import checkpoint_segment, integrate
    wl = workloads.WORKLOADS["disk_256x512"]
    grid = tg.Grid("disk", wl.n)
    plan = tg.Plan(grid, wl.diff, wl.reaction, wl.params, wl.tau, "fp32")
    x0 = plan.state_from_deviation(workloads.perturbation(wl)[None])
    tgt = torch.from_numpy(workloads.target_pattern(wl)).to("cuda", torch.float32)
    fwd_flops = sum(f for _, f in plan.chain())  # per step
    plan.set_route("generic")
    per_mode = [f for _, f in plan.chain()]
    segment = checkpoint_segment(x0, wl.steps)  # what integrate picks: 1 = every state kept
    res = {}

    def grad_run(adj, n_steps):
        w0 = x0.clone().requires_grad_(True)
        diff = torch.tensor([wl.diff], dtype=torch.float64, requires_grad=True)
        ab = torch.tensor([wl.params], dtype=torch.float64, requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outx = integrate(w0, grid, diff, ab, wl.tau, n_steps, precision="fp32",
                         w_ref=plan.reference, adjoint_precision=adj)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss = 0.5 * ((outx[0, 0] - tgt) ** 2).sum()
        loss.backward()
        torch.cuda.synchronize()
        return t1 - t0, time.perf_counter() - t1, w0.grad

    for adj in ("fp64", "same"):
        t0 = time.perf_counter()
        grad_run(adj, 20)  # builds and caches the plans, captures the graphs
        setup = time.perf_counter() - t0
        tf, tb, g = grad_run(adj, wl.steps)
        g2 = grad_run(adj, wl.steps)[2]
        # reverse sweep per step, in the adjoint plan's arithmetic: the
        # transposed chain (the forward's products once), the d-tangent chain
        # (the partial products S_k F of every op but the last, the tangent's
        # of every op but the first) and, with checkpoints, the recomputed
        # forward step
        ops = per_mode  # the adjoint runs the per-mode products
        rev_flops = fwd_flops + (2 * fwd_flops - ops[0] - ops[-1]) + (fwd_flops if segment > 1 else 0.0)
        res[adj] = {"forward_ms_per_step": tf * 1e3 / wl.steps, "gradient_ms_per_step": tb * 1e3 / wl.steps,
                    "gradient_over_forward": tb / tf, "first_call_s": setup,
                    "repeat_bitwise_equal": bool(torch.equal(g, g2)),
                    "forward_roofline": step_roofline(fwd_flops, tf / wl.steps, PEAK["fp32"], "forward step"),
                    "gradient_roofline": step_roofline(
                        rev_flops, tb / wl.steps, PEAK["fp64" if adj == "fp64" else "fp32"],
                        "reverse step (transposed and tangent chains%s)" % (
                            ", recomputed forward" if segment > 1 else "; every forward state kept"))}
    out["disk_256x512_gradient_400_steps"] = {
        "checkpoint_segment": segment,
        "fp32_forward_fp64_adjoint": res["fp64"], "fp32_forward_fp32_adjoint": res["same"]}
    return out


def profile_mode(tg, torch, w, pert, steps, route, tiles, precision="fp32"):
    """Direct launches of the step in a given launch configuration (for
    rocprofv3) and a copy of known size that calibrates the HBM byte counters.

    Workloads: the ball (64 x 64 x 128) and the cylinder (100^3, three
    species) take single steps of ``precision``; "sphere_batch" runs the 96
    sphere instances in grouped launches (FP32); "disk_256x512" runs the
    gradient workload (FP32 forward, FP64 reverse sweep) over ``steps`` steps."""
    if w.name == "sphere_256x512":
        big, small = workloads.WORKLOADS["sphere_256x512"], workloads.WORKLOADS["sphere_128x256"]
        prm = workloads.sphere_batch_params(big.batch + small.batch)
        plans, states = [], []
        for wl, rows in ((big, prm[:big.batch]), (small, prm[big.batch:])):
            diff = np.stack([np.ones(wl.batch), rows[:, 2]], axis=1)
            plan = tg.Plan(tg.Grid("sphere", wl.n), diff, "schnakenberg", rows[:, :2], wl.tau, "fp32", wl.batch)
            if route:  # the group autotuner's choice: a route shared by every plan
                plan.set_route(route)
            if tiles:  # and its tile widths (the same for both grids)
                plan.set_tiles([int(t) for t in tiles.split(",")])
            plans.append(plan)
            states.append(plan.state_from_deviation(workloads.batch_perturbations(wl)))
        info = tg.group_info(plans, states)
        print(f"configuration grouped={info['grouped']} route={plans[0].route} tiles={plans[0].tiles()}", flush=True)
        tg.group_run(plans, states, steps)
        desc = f"{steps} grouped FP32 steps of the 96-instance sphere batch"
    elif w.name == "disk_256x512":
        from paper_2604_11558_amd.autograd import integrate
        grid = tg.Grid("disk", w.n)
        plan = tg.Plan(grid, w.diff, w.reaction, w.params, w.tau, "fp32")
        x0 = plan.state_from_deviation(pert[None]).requires_grad_(True)
        tgt = torch.from_numpy(workloads.target_pattern(w)).to("cuda", torch.float32)
        out = integrate(x0, grid, torch.tensor([w.diff]), torch.tensor([w.params]), w.tau, steps,
                        precision="fp32", w_ref=plan.reference)
        loss = 0.5 * ((out[0, 0] - tgt) ** 2).sum()
        loss.backward()
        desc = f"{steps}-step FP32 forward and FP64 reverse sweep of the 256 x 512 disk gradient"
    else:
        grid = tg.Grid(w.geometry, w.n, w.extent)
        plan = tg.Plan(grid, w.diff, w.reaction, w.params, w.tau, precision)
        if route:
            plan.set_route(route)
        if tiles:
            plan.set_tiles([int(t) for t in tiles.split(",")])
        print(f"configuration {plan.route}:{','.join(map(str, plan.tiles()))}", flush=True)
        x = plan.state_from_deviation(pert)
        for _ in range(steps):
            plan.step(x)
        desc = f"{steps} steps of {w.name} ({precision})"
    torch.cuda.synchronize()
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"profiled {desc} and 5 copies of {COPY_BYTES} bytes", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=16)
    ap.add_argument("--workload", default="ball_64x64x128")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-other", action="store_true", help="skip the other workloads' lines")
    ap.add_argument("--profile", action="store_true",
                    help="only launch --steps FP32 steps and a calibration copy (for rocprofv3)")
    ap.add_argument("--route", default="", help="--profile: launch route (default: the plan's)")
    ap.add_argument("--tiles", default="", help="--profile: comma-separated tile widths")
    ap.add_argument("--precision", default="fp32", help="--profile: precision of the profiled steps")
    ap.add_argument("--fp32-config", default="",
                    help="route:tiles for the FP32 headline instead of the autotuner's choice "
                         "(e.g. fused:16,64; used to profile a fixed configuration)")
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
    if args.profile:
        profile_mode(tg, torch, w, pert, args.steps, args.route, args.tiles, args.precision)
        return
    grid = tg.Grid(w.geometry, w.n, w.extent)

    res = {}
    states = {}
    for prec in ("fp64", "fp32"):
        t0 = time.perf_counter()
        plan = tg.Plan(grid, w.diff, w.reaction, w.params, w.tau, prec)
        setup = time.perf_counter() - t0
        x = plan.state_from_deviation(pert)
        # launch configuration: route and tile widths chosen by the autotuner
        # (or given for FP32)
        if prec == "fp32" and args.fp32_config:
            rname, tl = args.fp32_config.split(":")
            plan.set_route(rname)
            plan.set_tiles([int(t) for t in tl.split(",")])
            tune = {"tiles": plan.tiles(), "us_per_step": None}
        else:
            tune = plan.autotune(x, iters=20)
        route = plan.route
        # timed region: W warm-up steps, then K steps replayed from the
        # captured graph (tg_run), synchronised on both sides
        sec = time_gpu_run(plan, x, args.steps, args.warmup, torch, label=prec)
        states[prec] = x.double().cpu().numpy()
        # per-launch durations: the same steps with direct launches and a HIP
        # event on the launch stream before every launch (tg_run_timed)
        xw = plan.state_from_deviation(pert)
        plan.run_timed(xw, args.warmup)
        torch.cuda.synchronize()
        launch_us = plan.run_timed(xw, args.steps)
        sec_direct = sum(launch_us) * 1e-6
        chain = plan.chain()
        flops = [f for _, f in chain]
        modes = [m for m, _ in chain]
        # average duration of each product launch, repeated back to back
        # between two HIP events (as in a step, except that the final update
        # is a store)
        bufs = [plan.state_from_deviation(pert), torch.empty_like(x), torch.empty_like(x)]
        op_times = []
        for i in range(len(chain)):
            src = bufs[0] if i == 0 else bufs[1 + (i - 1) % 2]
            dst = bufs[1 + i % 2]
            op_times.append(time_chain_op(plan, i, src, dst, 200, torch))
        del bufs
        dom = int(np.argmax(op_times))
        # the other routes for comparison
        other = {}
        for rname in ("fused", "generic", "fused_stencil_apart", "per_slice"):
            if rname == route:
                continue
            plan.set_route(rname)
            xg = plan.state_from_deviation(pert)
            plan.run(xg, args.warmup)
            other[rname] = time_gpu_run(plan, xg, min(args.steps, 200), 0, torch)
            del xg
        plan.set_route(route)
        res[prec] = dict(sec=sec, sec_direct=sec_direct, setup=setup, op_times=op_times,
                         step_launch_us=launch_us,
                         dom=dom, flops=flops, modes=modes, ref=plan.reference.copy(), route=route, other=other,
                         tiles=tune["tiles"], tune_us=tune["us_per_step"])
        del plan, x, xw
        torch.cuda.empty_cache()

    # split-bf16 precisions of the same step (fused route)
    bf = {}
    for prec in ("bf16x3", "bf16x2"):
        plan = tg.Plan(grid, w.diff, w.reaction, w.params, w.tau, prec)
        x = plan.state_from_deviation(pert)
        plan.autotune(x, iters=20)
        # the same W + K steps as the FP64 reference state
        sec = time_gpu_run(plan, x, args.steps, args.warmup, torch, label=prec)
        full = x.double().cpu().numpy() + plan.reference[:, :, None, None, None]
        bf[prec] = dict(sec=sec, full=full)
        del plan, x
        torch.cuda.empty_cache()

    dof = w.dof
    v32 = dof / res["fp32"]["sec"]
    v64 = dof / res["fp64"]["sec"]
    ref64 = states["fp64"] + res["fp64"]["ref"][:, :, None, None, None]
    full32 = states["fp32"] + res["fp32"]["ref"][:, :, None, None, None]
    err_32_64 = float(np.abs(full32 - ref64).max() / np.abs(ref64).max())
    dev64 = states["fp64"]
    err_32_64_dev = float(np.abs(full32 - ref64).max() / max(np.abs(dev64).max(), 1e-300))

    # time-discretisation error at tau by step doubling (first order: the
    # difference of the tau and tau/2 runs is about half the error of the tau
    # run), with the FP64 plan (held to the oracle at 1e-12) for speed; a
    # reduced precision counts as equally accurate below it
    nsteps = args.warmup + args.steps
    plan_h = tg.Plan(grid, w.diff, w.reaction, w.params, w.tau / 2, "fp64")
    xh = plan_h.state_from_deviation(pert)
    plan_h.run(xh, 2 * nsteps)
    half = xh.double().cpu().numpy() + plan_h.reference[:, :, None, None, None]
    del plan_h, xh
    t_err = 2.0 * float(np.abs(ref64 - half).max() / np.abs(ref64).max())

    r = res["fp32"]
    dom = r["dom"]
    if r["flops"][dom] > 0:  # a product launch: MFMA-bound
        achieved = r["flops"][dom] / r["op_times"][dom]
        roof = {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK["fp32"] / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK["fp32"], "flops_per_launch": r["flops"][dom],
                "kernel": f"launch {dom} of the {r['route']} route (leading mode {r['modes'][dom]})"}
    else:
        raise RuntimeError("a product launch without flops")
    key = f"{r['route']}:{dom}:{','.join(map(str, r['tiles']))}"
    roof["traffic"] = (TRAFFIC or {}).get(key) if TRAFFIC_DIGEST == kernel_sources_digest() else None
    roof["traffic_unit"] = "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
    # one read of the launch's input and one write of its output (the
    # plane-tail launch also reads the state it updates)
    roof["algorithmic_bytes_per_launch"] = dof * 4 * (3 if dom == len(r["flops"]) - 1 and dom > 0 else 2)
    roof["avg_launch_us"] = r["op_times"][dom] * 1e6
    roof["launch_key"] = key
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
                           "after_steps": args.warmup + args.steps,
                           "rel_err_vs_fp64_after_steps": float(np.abs(bf[p]["full"] - ref64).max()
                                                                / np.abs(ref64).max()),
                           "rel_err_vs_fp64_vs_max_deviation": float(np.abs(bf[p]["full"] - ref64).max()
                                                                     / max(np.abs(dev64).max(), 1e-300))}
                       for p in bf},
        # every speed-up over the plain FP64 step with its accuracy: the error
        # against the FP64 trajectory relative to the largest deviation from
        # the equilibrium (the part of the state the steps change)
        "speedups_vs_fp64_at_accuracy": {
            "fp32": {"speedup": v32 / v64, "rel_err_vs_max_deviation": err_32_64_dev},
            **{p: {"speedup": dof / bf[p]["sec"] / v64,
                   "rel_err_vs_max_deviation": float(np.abs(bf[p]["full"] - ref64).max()
                                                     / max(np.abs(dev64).max(), 1e-300))} for p in bf}},
        "rel_err_fp32_vs_fp64": {"after_steps": args.warmup + args.steps, "vs_max_state": err_32_64,
                                 "vs_max_deviation": err_32_64_dev},
        "time_discretisation_error": {"after_steps": nsteps, "vs_max_state": t_err,
                                      "method": "2 |W_tau - W_tau/2| / |W| (step doubling, FP64)"},
        "equal_accuracy": {"fp32": err_32_64 < t_err,
                           **{p: float(np.abs(bf[p]["full"] - ref64).max() / np.abs(ref64).max()) < t_err
                              for p in bf}},
        "route": res["fp32"]["route"],
        "autotuned": {p: {"route": res[p]["route"], "tiles": res[p]["tiles"]} for p in res},
        "ms_per_step_direct_launches_with_events": {p: res[p]["sec_direct"] * 1e3 for p in res},
        "launch_us_back_to_back": {p: [t * 1e6 for t in res[p]["op_times"]] for p in res},
        "launch_us_in_direct_steps": {p: res[p]["step_launch_us"] for p in res},
        "ms_per_step_other_routes": {p: {k: v * 1e3 for k, v in res[p]["other"].items()} for p in res},
        "plan_setup_s": {p: res[p]["setup"] for p in res},
        "graph_capture_s": dict(CAPTURE_S),
        "roofline": roof,
    }
    # step-level roofline (whole chain's flops in one step vs MFMA peak)
    step_flops = sum(res["fp32"]["flops"])
    out["step_roofline"] = {"flops_per_step": step_flops,
                            "fp32_frac": step_flops / res["fp32"]["sec"] / PEAK["fp32"],
                            "fp64_frac": step_flops / res["fp64"]["sec"] / PEAK["fp64"]}

    if not args.no_other:
        out["other_workloads"] = other_workloads(tg, torch, min(args.steps, 100))

    if not args.no_cpu:
        v_cpu, per_step, n_cpu, ws = cpu_baseline(w, pert, args.cpu_seconds)
        out["cpu_baseline"] = {"value": v_cpu, "unit": "dof-steps/s", "cores": blas_threads(),
                               "kind": "oracle", "host_cpu": cpu_model(), "host_cpu_count": os.cpu_count(),
                               "sample": f"{n_cpu} steps of {w.name} after one warm-up step (FP64 "
                                         f"NumPy/SciPy oracle), s/step = {per_step:.3f}"}
        # the same oracle on one BLAS thread, a short sample
        try:
            from threadpoolctl import threadpool_limits
            with threadpool_limits(limits=1):
                v1, per1, n1_, _ = cpu_baseline(w, pert, min(args.cpu_seconds, 4.0))
            out["cpu_baseline"]["one_thread"] = {"value": v1, "unit": "dof-steps/s",
                                                 "sample": f"{n1_} steps, s/step = {per1:.3f}"}
        except ImportError:
            pass
        # FP32 GPU path against the oracle on the same sample
        g32 = tg.Plan(grid, w.diff, w.reaction, w.params, w.tau, "fp32")
        x = g32.state_from_deviation(pert)
        g32.run(x, n_cpu + 1)
        got = x.double().cpu().numpy() + g32.reference[:, :, None, None, None]
        out["rel_err_fp32_vs_oracle"] = {"after_steps": n_cpu + 1,
                                         "vs_max_state": float(np.abs(got[0] - ws).max() / np.abs(ws).max())}
    print(json.dumps(out, default=lambda o: o.item() if hasattr(o, "item") else str(o)))


if __name__ == "__main__":
    main()
