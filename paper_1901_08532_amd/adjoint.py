"""Differentiable shared-step Hermite-6 integration on the GPU.

``hermite_shared_run(x0, v0, m, ...)`` returns the final positions after the
start-up passes and ``nsteps`` shared steps of length ``dt``, as a
``torch.autograd.Function``: gradients of any loss on the final positions
with respect to the initial positions, velocities and masses come from the
hand-written adjoint kernels of libh6 (h6_correct_shared_vjp,
h6_evaluate_vjp, h6_predict_dt_vjp, h6_init_forces_vjp), never from torch
autograd of the arithmetic.

Memory: the forward pass keeps the full state every ``checkpoint`` steps.
The backward pass walks the segments from last to first; for each it
replays the segment's steps forward from its checkpoint (bitwise the same
kernels, so the same values) keeping the predicted states, then applies,
step by step in reverse, the transpose of the corrector, the VJP of the
evaluation at the kept predicted state, and the transpose of the predictor.
Finally the start-up passes are reversed. This module only sequences
library calls and allocates work arrays.
"""

from __future__ import annotations

import torch

from . import h6


class _HermiteSharedRun(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x0, v0, m, lib_ctx, dt, nsteps, checkpoint):
        n = x0.shape[0]
        dev = x0.device
        S = torch.zeros((18, n), dtype=torch.float64, device=dev)
        S[0:3] = x0.detach().T
        S[3:6] = v0.detach().T
        mm = m.detach().contiguous()
        P = torch.empty((9, n), dtype=torch.float64, device=dev)
        F = torch.empty((9, n), dtype=torch.float64, device=dev)
        lib_ctx.h6_init_forces(S, mm)
        ckpts = []
        for step in range(nsteps):
            if step % checkpoint == 0:
                ckpts.append(S.clone())
            lib_ctx.h6_shared_steps(S, mm, P, F, dt, 1)
        ctx.lib_ctx = lib_ctx
        ctx.dt = dt
        ctx.nsteps = nsteps
        ctx.checkpoint = checkpoint
        ctx.ckpts = ckpts if nsteps > 0 else [S.clone()]
        ctx.save_for_backward(mm)
        return S[0:3].T.contiguous()

    @staticmethod
    def backward(ctx, gx):
        (mm,) = ctx.saved_tensors
        lc, dt, k = ctx.lib_ctx, ctx.dt, ctx.checkpoint
        n = mm.shape[0]
        dev = mm.device
        cot = torch.zeros((18, n), dtype=torch.float64, device=dev)
        cot[0:3] = gx.T
        gm = torch.zeros(n, dtype=torch.float64, device=dev)
        CF = torch.empty((9, n), dtype=torch.float64, device=dev)
        CP = torch.empty((9, n), dtype=torch.float64, device=dev)
        F = torch.empty((9, n), dtype=torch.float64, device=dev)
        for seg in reversed(range(len(ctx.ckpts) if ctx.nsteps > 0 else 0)):
            S = ctx.ckpts[seg].clone()
            count = min(k, ctx.nsteps - seg * k)
            preds = [torch.empty((9, n), dtype=torch.float64, device=dev) for _ in range(count)]
            for st in range(count):
                lc.h6_predict_dt(S, mm, dt, preds[st])
                lc.h6_evaluate(preds[st], mm, None, n, h6.H6_FP64, F)
                lc.h6_correct_shared(S, mm, F, dt)
            for st in reversed(range(count)):
                lc.h6_correct_shared_vjp(cot, gm, CF, dt)
                lc.h6_evaluate_vjp(preds[st], mm, CF, CP, gm)
                lc.h6_predict_dt_vjp(cot, gm, CP, dt)
        lc.h6_init_forces_vjp(ctx.ckpts[0], mm, cot, gm)
        return cot[0:3].T.contiguous(), cot[3:6].T.contiguous(), gm, None, None, None, None


def hermite_shared_run(x0, v0, m, lib_ctx: h6.Context, dt: float, nsteps: int,
                       checkpoint: int = 8):
    """Final positions (n, 3) after start-up and nsteps shared steps of dt.

    x0, v0: (n, 3) float64 CUDA tensors; m: (n,) float64 CUDA tensor.
    Differentiable with respect to all three.
    """
    if checkpoint < 1:
        raise ValueError("checkpoint must be >= 1")
    return _HermiteSharedRun.apply(x0, v0, m, lib_ctx, float(dt), int(nsteps), int(checkpoint))
