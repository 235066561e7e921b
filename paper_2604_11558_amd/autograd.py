"""Differentiable integration with the hand-written GPU adjoint.

``integrate(...)`` runs ``n_steps`` split exponential Euler steps on the GPU
and returns the final state; its backward pass applies ``tg_adjoint_step``
in reverse with sqrt(T) checkpointing: the forward keeps one state every
``segment`` steps, and the backward recomputes each segment from its
checkpoint (storing that segment's states) before walking it in reverse,
so memory is O(sqrt(T)) states and the forward is recomputed once.

Gradients are returned for the initial state (a deviation from the fixed
reference state ``w_ref``), the diffusion coefficients ``diff``
[batch, n_species] and the reaction constants a, b ([batch, 2]: they enter
the first two species' reactions additively).  The reference state is not
differentiated.

The reverse sweep multiplies the rounding of tau S^T lambda by
tau d M^T, whose norm grows like 1/h^2 and, near the axis and the poles,
like 1/r^2 and 1/sin^2; in FP32 that costs up to ~1e-3 of relative
accuracy in lambda on stiff grids.  By default the adjoint steps therefore
run on an FP64 plan of the same problem, fed with the recomputed
lower-precision states (``adjoint_precision="fp64"``); ``"same"`` keeps
the forward plan's arithmetic.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import Grid, Plan


class SplitEEFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, w0, diff, ab, grid, reaction, extra_params, w_ref, tau, precision, n_steps, segment,
                adjoint_precision):
        batch = diff.shape[0]
        params = np.concatenate([ab.detach().cpu().numpy().reshape(batch, 2),
                                 np.asarray(extra_params, float).reshape(batch, -1)], axis=1) \
            if extra_params is not None else ab.detach().cpu().numpy().reshape(batch, 2)
        plan = Plan(grid, diff.detach().cpu().numpy(), reaction, params, tau, precision, batch,
                    w_ref=w_ref)
        x = w0.detach().to(plan.dtype).contiguous().clone()
        ckpts = []
        done = 0
        while done < n_steps:
            ckpts.append(x.clone())
            k = min(segment, n_steps - done)
            plan.run(x, k)
            done += k
        ctx.plan = plan
        ctx.adj_plan = plan
        if adjoint_precision == "fp64" and precision != "fp64":
            ctx.adj_plan = Plan(grid, diff.detach().cpu().numpy(), reaction, params, tau, "fp64", batch,
                                w_ref=plan.reference)
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
        for k in range(len(ckpts) - 1, -1, -1):
            start = k * ctx.segment
            length = min(ctx.segment, ctx.n_steps - start)
            states = [ckpts[k]]
            x = ckpts[k].clone()
            for _ in range(length - 1):
                plan.step(x)
                states.append(x.clone())
            for st in reversed(states):
                adj.adjoint_step(st.to(adj.dtype).contiguous(), lam, grad)
        torch.cuda.synchronize()
        g = grad.cpu().numpy()
        g_diff = torch.from_numpy(g[:nslab].reshape(dshape))
        src = g[nslab:].reshape(plan.batch, plan.n_species)
        g_ab = torch.from_numpy(src[:, :2].copy()).reshape(abshape)
        return lam.to(w_dtype), g_diff, g_ab, None, None, None, None, None, None, None, None, None


def integrate(w0, grid: Grid, diff, ab, tau: float, n_steps: int, reaction: str = "schnakenberg",
              extra_params=None, w_ref=None, precision: str = "fp64", segment: int = 0,
              adjoint_precision: str = "fp64"):
    """Final state after ``n_steps`` steps, differentiable in (w0, diff, ab).

    w0: device tensor of the plan's state shape (deviation from ``w_ref``);
    diff: CPU float64 tensor [batch, n_species]; ab: CPU float64 tensor
    [batch, 2] (constants a, b); extra_params: further reaction constants
    (not differentiated); w_ref: [batch, n_species] reference state, by
    default the equilibrium at the given (a, b), held fixed; segment:
    steps between checkpoints (0: ceil(sqrt(n_steps))); adjoint_precision:
    "fp64" or "same" (the forward plan's arithmetic).
    """
    if adjoint_precision not in ("fp64", "same"):
        raise ValueError("adjoint_precision must be 'fp64' or 'same'")
    if segment <= 0:
        segment = max(1, int(math.ceil(math.sqrt(n_steps))))
    diff = torch.as_tensor(diff, dtype=torch.float64)
    ab = torch.as_tensor(ab, dtype=torch.float64)
    if diff.dim() == 1:
        diff = diff[None, :]
    if ab.dim() == 1:
        ab = ab[None, :]
    return SplitEEFunction.apply(w0, diff, ab, grid, reaction, extra_params, w_ref, float(tau), precision,
                                 int(n_steps), int(segment), adjoint_precision)
