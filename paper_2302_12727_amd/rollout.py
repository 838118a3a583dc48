"""Differentiable RT rollout with step checkpointing.

`RTRollout.apply(L, U0, rt, steps, ckpt_every)` runs `steps` RT steps
(injection -> gradient -> transport) on the library context `rt` and returns
the final state.  Its backward walks the checkpoint segments in reverse: each
segment is recomputed from its checkpoint (keeping the gradient records and
the unguarded updated states of its steps), then rt_adjoint is applied step
by step, accumulating dLoss/dL and carrying dLoss/dU back to U0.  The last
segment's records are kept by the forward itself when a backward will follow,
so that segment is never recomputed.

All arithmetic runs in the library's HIP kernels; this module only orders the
calls and keeps the checkpoints (device tensors).
"""
from __future__ import annotations

import torch


class RolloutBuffers:
    """Device buffers of a rollout of `steps` steps with checkpoints every
    `ckpt_every`, allocated once and reused by every call that passes them:
    the working and spare states, the gradient record of a step, the
    checkpoints, and the records of one segment (the gradient records and
    unguarded states the forward keeps for the last segment and the backward's
    recomputes refill).  With them a rollout allocates only its output and the
    cotangents.  Calls sharing one set must not overlap."""

    def __init__(self, rt, steps: int, ckpt_every: int):
        K = max(1, int(ckpt_every))
        self.steps, self.K = int(steps), K
        self.U, self.Ub, self.UD = rt.state(), rt.state(), rt.grad_buffer()
        self.ckpts = {s: rt.state() for s in range(0, max(1, self.steps), K)}
        self.rec = [(rt.grad_buffer(), rt.state()) for _ in range(min(K, max(1, self.steps)))]


class RTRollout(torch.autograd.Function):

    @staticmethod
    def forward(ctx, L, U0, rt, steps: int, ckpt_every: int, keep_last: bool = False,
                bufs: RolloutBuffers = None):
        K = max(1, int(ckpt_every))
        if bufs is not None and (bufs.steps != steps or bufs.K != K):
            raise ValueError("RolloutBuffers made for another rollout length or checkpointing")
        if bufs is None:
            U, Ub, UD = U0.detach().clone(), torch.empty_like(U0), rt.grad_buffer()
            ckpts = {0: U.clone()}
        else:
            U, Ub, UD = bufs.U, bufs.Ub, bufs.UD
            U.copy_(U0.detach())
            ckpts = bufs.ckpts
            ckpts[0].copy_(U)
        Ld = L.detach()
        s_last = ((steps - 1) // K) * K if steps > 0 else 0
        last = []
        for n in range(steps):
            if rt.S:
                rt.rt_inject(U, Ld)
            if keep_last and n >= s_last:
                if bufs is None:
                    UDk, Uu = rt.grad_buffer(), torch.empty_like(U)
                else:
                    UDk, Uu = bufs.rec[n - s_last]
                rt.rt_gradient(U, UDk)
                rt.rt_transport(UDk, U_out=Ub, U_unguarded=Uu)
                last.append((UDk, Uu))
            else:
                rt.rt_gradient(U, UD)
                rt.rt_transport(UD, U_out=Ub)
            U, Ub = Ub, U
            if (n + 1) % K == 0 and n + 1 < steps:
                if bufs is None:
                    ckpts[n + 1] = U.clone()
                else:
                    ckpts[n + 1].copy_(U)
        ctx.rt, ctx.steps, ctx.K, ctx.ckpts, ctx.bufs = rt, steps, K, ckpts, bufs
        ctx.last = (s_last, last) if keep_last else None
        ctx.save_for_backward(Ld)
        return U.clone()

    @staticmethod
    def backward(ctx, gU):
        (L,) = ctx.saved_tensors
        rt, steps, K, bufs = ctx.rt, ctx.steps, ctx.K, ctx.bufs
        lam = gU.detach().to(rt.sdtype).contiguous().clone()
        dLdL = torch.zeros((max(rt.S, 1), rt.G), dtype=torch.float64, device=lam.device)
        for s0 in reversed(range(0, steps, K)):
            s1 = min(s0 + K, steps)
            if ctx.last is not None and ctx.last[0] == s0:
                rec = ctx.last[1]
                ctx.last = None
            else:
                # the last segment's records, once consumed, take the recompute
                if bufs is None:
                    U, Ub = ctx.ckpts[s0].clone(), None
                else:
                    U, Ub = bufs.U, bufs.Ub
                    U.copy_(ctx.ckpts[s0])
                if Ub is None:
                    Ub = torch.empty_like(U)
                rec = []
                for n in range(s0, s1):
                    if rt.S:
                        rt.rt_inject(U, L)
                    if bufs is None:
                        UD, Uu = rt.grad_buffer(), torch.empty_like(U)
                    else:
                        UD, Uu = bufs.rec[n - s0]
                    rt.rt_gradient(U, UD)
                    rt.rt_transport(UD, U_out=Ub, U_unguarded=Uu)
                    U, Ub = Ub, U
                    rec.append((UD, Uu))
            for UD, Uu in reversed(rec):
                rt.rt_adjoint(None, L, lam, lam=lam, UD=UD, U_unguarded=Uu,
                              dL_dL=dLdL if rt.S else None)
            del rec
        ctx.last = None
        gL = dLdL[:rt.S] if rt.S else None
        return gL, lam, None, None, None, None, None


def rollout(rt, L, U0, steps: int, ckpt_every: int = 5, bufs: RolloutBuffers = None):
    """Differentiable final state after `steps` RT steps (see RTRollout);
    `bufs` (a RolloutBuffers of the same length and checkpointing) makes the
    forward and backward reuse preallocated device buffers."""
    keep = torch.is_grad_enabled() and (L.requires_grad or U0.requires_grad)
    return RTRollout.apply(L, U0, rt, steps, ckpt_every, keep, bufs)
