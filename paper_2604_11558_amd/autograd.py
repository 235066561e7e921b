"""Differentiable integration with the hand-written GPU adjoint.

``integrate(...)`` runs ``n_steps`` split exponential Euler steps on the GPU
and returns the final state; its backward pass applies ``tg_adjoint_step``
in reverse.  When the T states fit a memory budget (at most a quarter of
the free device memory, and 8 GiB) the forward keeps every one of them and
the reverse sweep recomputes nothing; otherwise it checkpoints: the forward
keeps one state every ``segment`` steps (sqrt(T) by default), and the
backward recomputes each segment from its checkpoint (storing that
segment's states) before walking it in reverse, so memory is O(sqrt(T))
states and the forward is recomputed once.

Gradients are returned for the initial state (a deviation from the fixed
reference state ``w_ref``), the diffusion coefficients ``diff``
[batch, n_species] and the reaction constants a, b ([batch, 2]).  In the
plain Schnakenberg and three-species kinetics a and b are additive sources
of the first two species; in the alpha_1-scaled Schnakenberg kinetics of
Section 5.3 they enter as gamma a and gamma b (gamma = alpha_1, the third
reaction constant), so their gradient carries that factor.  The reference
state is not differentiated: it must be given explicitly when ``ab``
requires a gradient (the default reference, the equilibrium at (a, b),
would make the initial absolute state depend on (a, b) in a way the
reverse sweep does not follow).

The reverse sweep multiplies the rounding of tau S^T lambda by
tau d M^T, whose norm grows like 1/h^2 and, near the axis and the poles,
like 1/r^2 and 1/sin^2; in FP32 that costs up to ~1e-3 of relative
accuracy in lambda on stiff grids.  By default the adjoint steps therefore
run on an FP64 plan of the same problem, fed with the recomputed
lower-precision states (``adjoint_precision="fp64"``); ``"same"`` keeps
the forward plan's arithmetic.

Plans are built once per problem (grid, coefficients, constants, reference,
tau, precision), the forward plan autotuned on the first call's initial
state, and kept in a small cache, so repeated calls (an optimiser loop)
spend no time on set-up.
"""
from __future__ import annotations

import math
from collections import OrderedDict

import numpy as np
import torch

from . import Grid, Plan

_PLAN_CACHE: "OrderedDict[tuple, Plan]" = OrderedDict()
_PLAN_CACHE_SIZE = 4


def cached_plan(grid: Grid, diff: np.ndarray, reaction: str, params: np.ndarray, tau: float,
                precision: str, batch: int, w_ref, tune_state=None) -> Plan:
    """A plan for this problem, built on first use (and autotuned on a copy
    of ``tune_state`` if given) and then reused."""
    wr = None if w_ref is None else np.ascontiguousarray(
        np.broadcast_to(np.asarray(w_ref, dtype=np.float64), diff.shape))
    key = (id(grid), grid.geometry, grid.n, grid.extent, diff.tobytes(), diff.shape, reaction,
           params.tobytes(), params.shape, float(tau), precision, int(batch),
           None if wr is None else wr.tobytes())
    plan = _PLAN_CACHE.get(key)
    if plan is not None and plan.grid is grid:
        _PLAN_CACHE.move_to_end(key)
        return plan
    plan = Plan(grid, diff, reaction, params, tau, precision, batch, w_ref=wr)
    if tune_state is not None:
        plan.autotune(tune_state.detach().to(plan.dtype).contiguous(), iters=10)
    _PLAN_CACHE[key] = plan
    while len(_PLAN_CACHE) > _PLAN_CACHE_SIZE:
        _PLAN_CACHE.popitem(last=False)
    return plan


def clear_plan_cache() -> None:
    _PLAN_CACHE.clear()


_STORE_ALL_CAP = 8 << 30


def checkpoint_segment(w0, n_steps: int) -> int:
    """Steps between checkpoints: 1 (keep every state) when n_steps states
    of w0's size, kept in FP64, fit min(8 GiB, a quarter of the free device
    memory), else ceil(sqrt(n_steps))."""
    need = int(n_steps) * w0.numel() * 8
    free, _ = torch.cuda.mem_get_info(w0.device)
    if need <= min(_STORE_ALL_CAP, free // 4):
        return 1
    return max(1, int(math.ceil(math.sqrt(n_steps))))


class SplitEEFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, w0, diff, ab, grid, reaction, extra_params, w_ref, tau, precision, n_steps, segment,
                adjoint_precision):
        batch = diff.shape[0]
        ab_np = ab.detach().cpu().numpy().reshape(batch, 2)
        params = np.concatenate([ab_np, np.asarray(extra_params, float).reshape(batch, -1)], axis=1) \
            if extra_params is not None else ab_np
        diff_np = np.ascontiguousarray(diff.detach().cpu().numpy())
        params = np.ascontiguousarray(params)
        plan = cached_plan(grid, diff_np, reaction, params, tau, precision, batch, w_ref, tune_state=w0)
        # steps run on one buffer per plan, so the graphs tg_run replays are
        # captured once for it rather than once per call
        x = getattr(plan, "_autograd_state", None)
        if x is None or x.shape != w0.shape or x.device != w0.device:
            x = torch.empty(w0.shape, dtype=plan.dtype, device=w0.device)
            plan._autograd_state = x
        x.copy_(w0.detach())
        wide = adjoint_precision == "fp64" and plan.dtype != torch.float64
        if segment == 1:  # every state, in one allocation, in the reverse sweep's precision
            hist = torch.empty((n_steps,) + tuple(x.shape), dtype=torch.float64 if wide else x.dtype,
                               device=x.device)
            plan.run_history(x, n_steps, hist)
            ckpts = list(hist.unbind(0))
        else:
            ckpts = []
            done = 0
            while done < n_steps:
                ckpts.append(x.clone())
                k = min(segment, n_steps - done)
                plan.run(x, k)
                done += k
        x = x.clone()
        ctx.plan = plan
        ctx.adj_plan = plan
        if adjoint_precision == "fp64" and precision != "fp64":
            ctx.adj_plan = cached_plan(grid, diff_np, reaction, params, tau, "fp64", batch, plan.reference)
        ctx.gamma = params[:, 2].copy() if reaction == "schnakenberg_scaled" else None
        ctx.ckpts = ckpts
        ctx.n_steps = n_steps
        ctx.segment = segment
        ctx.shapes = (w0.dtype, diff.shape, ab.shape)
        return x

    @staticmethod
    def backward(ctx, grad_out):
        plan, adj, ckpts = ctx.plan, ctx.adj_plan, ctx.ckpts
        w_dtype, dshape, abshape = ctx.shapes
        lam = grad_out.detach().to(adj.dtype).contiguous().clone()
        nslab = plan.batch * plan.n_species
        grad = torch.zeros(2 * nslab, dtype=torch.float64, device=lam.device)
        # one segment's states, reused for every segment; when the reverse
        # sweep runs in another precision, one conversion buffer
        seg_states = [torch.empty_like(ckpts[0]) for _ in range(min(ctx.segment, ctx.n_steps))]
        conv = None if adj.dtype == plan.dtype else torch.empty(ckpts[0].shape, dtype=adj.dtype,
                                                                 device=lam.device)
        for k in range(len(ckpts) - 1, -1, -1):
            start = k * ctx.segment
            length = min(ctx.segment, ctx.n_steps - start)
            if length == 1:  # a stored state: nothing to recompute
                st = ckpts[k]
                if st.dtype != adj.dtype:
                    conv.copy_(st)
                    st = conv
                adj.adjoint_step(st, lam, grad)
                continue
            seg_states[0].copy_(ckpts[k])
            for i in range(1, length):
                seg_states[i].copy_(seg_states[i - 1])
                plan.step(seg_states[i])
            for i in range(length - 1, -1, -1):
                st = seg_states[i]
                if conv is not None:
                    conv.copy_(st)
                    st = conv
                adj.adjoint_step(st, lam, grad)
        torch.cuda.synchronize()
        g = grad.cpu().numpy()
        g_diff = torch.from_numpy(g[:nslab].reshape(dshape))
        src = g[nslab:].reshape(plan.batch, plan.n_species)[:, :2].copy()
        if ctx.gamma is not None:  # the kinetics carry gamma a and gamma b
            src *= ctx.gamma[:, None]
        g_ab = torch.from_numpy(src).reshape(abshape)
        return lam.to(w_dtype), g_diff, g_ab, None, None, None, None, None, None, None, None, None


def integrate(w0, grid: Grid, diff, ab, tau: float, n_steps: int, reaction: str = "schnakenberg",
              extra_params=None, w_ref=None, precision: str = "fp64", segment: int = 0,
              adjoint_precision: str = "fp64"):
    """Final state after ``n_steps`` steps, differentiable in (w0, diff, ab).

    w0: device tensor of the plan's state shape (deviation from ``w_ref``);
    diff: CPU float64 tensor [batch, n_species]; ab: CPU float64 tensor
    [batch, 2] (constants a, b); extra_params: further reaction constants
    (not differentiated; for "schnakenberg_scaled" the third constant is
    gamma = alpha_1); w_ref: [batch, n_species] reference state, held fixed
    (required when ``ab`` requires a gradient; otherwise it defaults to the
    equilibrium at the given (a, b)); segment: steps between checkpoints
    (1: every state kept, no recompute; 0: 1 when the n_steps states fit the
    memory budget, else ceil(sqrt(n_steps))); adjoint_precision: "fp64" or
    "same" (the forward plan's arithmetic).
    """
    if adjoint_precision not in ("fp64", "same"):
        raise ValueError("adjoint_precision must be 'fp64' or 'same'")
    if segment <= 0:
        segment = checkpoint_segment(w0, n_steps)
    if w_ref is None and isinstance(ab, torch.Tensor) and ab.requires_grad:
        raise ValueError("integrate: give w_ref explicitly when ab requires a gradient (the reference "
                         "state is held fixed by the reverse sweep)")
    diff = torch.as_tensor(diff, dtype=torch.float64)
    ab = torch.as_tensor(ab, dtype=torch.float64)
    if diff.dim() == 1:
        diff = diff[None, :]
    if ab.dim() == 1:
        ab = ab[None, :]
    return SplitEEFunction.apply(w0, diff, ab, grid, reaction, extra_params, w_ref, float(tau), precision,
                                 int(n_steps), int(segment), adjoint_precision)
