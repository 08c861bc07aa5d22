"""Differentiable Hermite-6 integration on the GPU.

``hermite_shared_run(x0, v0, m, ...)`` returns the final positions (and,
on request, velocities) after the start-up passes and ``nsteps`` shared
steps of length ``dt``, as a ``torch.autograd.Function``: gradients of any
loss on the final state with respect to the initial positions, velocities
and masses come from the hand-written adjoint kernels of libh6
(h6_correct_shared_vjp, h6_evaluate_vjp, h6_predict_dt_vjp,
h6_init_forces_vjp), never from torch autograd of the arithmetic.

``hermite_block_run`` does the same for block time steps up to a given
time: the steps are chosen by the forward run and then held fixed (the
gradient does not flow through the step choice), and each block is
reversed with h6_correct_vjp, h6_evaluate_vjp_active (2 n_act n pairs) and
h6_predict_vjp. ``system_energy`` is the total energy as a differentiable
function of positions, velocities and masses (h6_energy forward;
h6_evaluate and h6_potential for its gradient), for energy-based losses.

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
        return S[0:3].T.contiguous(), S[3:6].T.contiguous()

    @staticmethod
    def backward(ctx, gx, gv):
        (mm,) = ctx.saved_tensors
        lc, dt, k = ctx.lib_ctx, ctx.dt, ctx.checkpoint
        n = mm.shape[0]
        dev = mm.device
        cot = torch.zeros((18, n), dtype=torch.float64, device=dev)
        cot[0:3] = gx.T
        cot[3:6] = gv.T
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
                       checkpoint: int = 8, return_velocities: bool = False):
    """Final positions (n, 3) after start-up and nsteps shared steps of dt;
    with return_velocities, the pair (positions, velocities).

    x0, v0: (n, 3) float64 CUDA tensors; m: (n,) float64 CUDA tensor.
    Differentiable with respect to all three.
    """
    if checkpoint < 1:
        raise ValueError("checkpoint must be >= 1")
    xT, vT = _HermiteSharedRun.apply(x0, v0, m, lib_ctx, float(dt), int(nsteps), int(checkpoint))
    return (xT, vT) if return_velocities else xT


class _HermiteBlockRun(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x0, v0, m, lib_ctx, t_end, eta, lev_min, lev_max, eta_s, checkpoint):
        n = x0.shape[0]
        dev = x0.device
        S = torch.zeros((18, n), dtype=torch.float64, device=dev)
        S[0:3] = x0.detach().T
        S[3:6] = v0.detach().T
        mm = m.detach().contiguous()
        T = torch.zeros((2, n), dtype=torch.int64, device=dev)
        P = torch.empty((9, n), dtype=torch.float64, device=dev)
        F = torch.empty((9, n), dtype=torch.float64, device=dev)
        act = torch.empty(n, dtype=torch.int32, device=dev)
        lib_ctx.h6_init_forces(S, mm)
        lib_ctx.h6_initial_steps(S, mm, T, eta_s, lev_min, lev_max)
        S0 = S.clone()
        ckpts = []
        seq = []  # the block sequence: (time, active count, active particles)
        blocks = 0
        while True:
            tn, na = lib_ctx.h6_next_block(S, mm, T, act)
            if tn > t_end:
                break
            if blocks % checkpoint == 0:
                ckpts.append((S.clone(), T.clone()))
            seq.append((tn, na, act[:na].clone()))
            _block(lib_ctx, S, mm, T, P, F, act, tn, na, eta, lev_min, lev_max)
            blocks += 1
        rc = lib_ctx.h6_check_status()
        if rc == h6.H6_ENONFINITE:  # H6_EDTMIN only reports steps clamped at 2^-lev_max
            raise h6.H6Error(rc, "block run")
        ctx.lib_ctx = lib_ctx
        ctx.params = (eta, lev_min, lev_max, checkpoint, blocks)
        ctx.ckpts = ckpts
        ctx.seq = seq
        ctx.S0 = S0
        ctx.save_for_backward(mm)
        return S[0:3].T.contiguous(), S[3:6].T.contiguous()

    @staticmethod
    def backward(ctx, gx, gv):
        (mm,) = ctx.saved_tensors
        lc = ctx.lib_ctx
        eta, lev_min, lev_max, k, blocks = ctx.params
        n = mm.shape[0]
        dev = mm.device
        cot = torch.zeros((18, n), dtype=torch.float64, device=dev)
        cot[0:3] = gx.T
        cot[3:6] = gv.T
        gm = torch.zeros(n, dtype=torch.float64, device=dev)
        F = torch.empty((9, n), dtype=torch.float64, device=dev)
        CF = torch.empty((9, n), dtype=torch.float64, device=dev)
        CP = torch.empty((9, n), dtype=torch.float64, device=dev)
        for seg in reversed(range(len(ctx.ckpts))):
            # replay the segment from its checkpoint along the recorded block
            # sequence (the same kernels: the same values), with no host
            # round trip per block
            S, T = (t.clone() for t in ctx.ckpts[seg])
            recs = []
            for tn, na, a_idx in ctx.seq[seg * k: min(blocks, (seg + 1) * k)]:
                T_old = T.clone()
                P = torch.empty((9, n), dtype=torch.float64, device=dev)
                _block(lc, S, mm, T, P, F, a_idx, tn, na, eta, lev_min, lev_max)
                recs.append((tn, na, a_idx, T_old, P))
            for tn, na, a_idx, T_old, P in reversed(recs):
                lc.h6_correct_vjp(cot, gm, a_idx, na, T_old[1], CF)
                CP.zero_()
                lc.h6_evaluate_vjp_active(P, mm, a_idx, na, CF, CP, gm)
                lc.h6_predict_vjp(cot, gm, T_old[0], tn, CP)
        lc.h6_init_forces_vjp(ctx.S0, mm, cot, gm)
        return (cot[0:3].T.contiguous(), cot[3:6].T.contiguous(), gm,
                None, None, None, None, None, None, None)


def _block(lc, S, m, T, P, F, act, tn, na, eta, lev_min, lev_max):
    """One block step at time tn over the na particles in act: predict all,
    evaluate the active set, correct it (its new steps chosen here)."""
    lc.h6_predict(S, m, T, tn, P)
    lc.h6_evaluate(P, m, act, na, h6.H6_FP64, F)
    lc.h6_correct(S, m, T, act, na, F, tn, eta, lev_min, lev_max)


def hermite_block_run(x0, v0, m, lib_ctx: h6.Context, t_end_ticks: int, eta: float = 0.4,
                      lev_min: int = 4, lev_max: int = 30, eta_s: float = 0.1,
                      checkpoint: int = 16):
    """Final (positions, velocities), each (n, 3), after the start-up passes
    and every block step up to time t_end_ticks (blocks with a later time
    are not taken; all particles are synchronised when t_end_ticks is a
    multiple of the largest step 2^-lev_min).

    Steps: initial ones from the 4th-order criterion (eta_s), then the
    6th-order block rule (eta, levels lev_min..lev_max), as h6_block_step.
    The gradient treats every step length as fixed. The forward pass keeps
    the state every `checkpoint` blocks and the block sequence (each block's
    time and active particles); the backward pass replays each segment from
    its checkpoint along that sequence (the same kernels, so the same
    values, and no host round trip per block) and reverses its blocks.
    """
    if checkpoint < 1:
        raise ValueError("checkpoint must be >= 1")
    return _HermiteBlockRun.apply(x0, v0, m, lib_ctx, int(t_end_ticks), float(eta), int(lev_min),
                                  int(lev_max), float(eta_s), int(checkpoint))


class _SystemEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, v, m, lib_ctx):
        n = x.shape[0]
        S = torch.zeros((18, n), dtype=torch.float64, device=x.device)
        S[0:3] = x.detach().T
        S[3:6] = v.detach().T
        mm = m.detach().contiguous()
        k, w, _ = lib_ctx.h6_energy(S, mm)
        ctx.lib_ctx = lib_ctx
        ctx.save_for_backward(S, mm)
        return torch.tensor(k + w, dtype=torch.float64, device=x.device)

    @staticmethod
    def backward(ctx, ge):
        S, mm = ctx.saved_tensors
        n = mm.shape[0]
        # dE/dx, dE/dv, dE/dm times the cotangent, all on the device (h6_energy_vjp)
        GS = torch.empty((18, n), dtype=torch.float64, device=S.device)
        gm = torch.empty(n, dtype=torch.float64, device=S.device)
        ge = ge.detach().to(device=S.device, dtype=torch.float64).contiguous()
        ctx.lib_ctx.h6_energy_vjp(S, mm, ge, GS, gm)
        return GS[0:3].T, GS[3:6].T, gm, None


def system_energy(x, v, m, lib_ctx: h6.Context):
    """Total energy (kinetic plus softened potential, the context's eps) of
    positions x, velocities v (n, 3) and masses m (n,), as a 0-d tensor,
    differentiable with respect to all three."""
    return _SystemEnergy.apply(x, v, m, lib_ctx)
