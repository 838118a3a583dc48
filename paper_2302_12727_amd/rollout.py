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


class RTRollout(torch.autograd.Function):

    @staticmethod
    def forward(ctx, L, U0, rt, steps: int, ckpt_every: int, keep_last: bool = False):
        K = max(1, int(ckpt_every))
        U = U0.detach().clone()
        Ub = torch.empty_like(U)
        UD = rt.grad_buffer()
        ckpts = {0: U.clone()}
        Ld = L.detach()
        s_last = ((steps - 1) // K) * K if steps > 0 else 0
        last = []
        for n in range(steps):
            if rt.S:
                rt.rt_inject(U, Ld)
            if keep_last and n >= s_last:
                UD = rt.rt_gradient(U)
                Uu = torch.empty_like(U)
                rt.rt_transport(UD, U_out=Ub, U_unguarded=Uu)
                last.append((UD, Uu))
            else:
                rt.rt_gradient(U, UD)
                rt.rt_transport(UD, U_out=Ub)
            U, Ub = Ub, U
            if (n + 1) % K == 0 and n + 1 < steps:
                ckpts[n + 1] = U.clone()
        ctx.rt, ctx.steps, ctx.K, ctx.ckpts = rt, steps, K, ckpts
        ctx.last = (s_last, last) if keep_last else None
        ctx.save_for_backward(Ld)
        return U.clone()

    @staticmethod
    def backward(ctx, gU):
        (L,) = ctx.saved_tensors
        rt, steps, K = ctx.rt, ctx.steps, ctx.K
        lam = gU.detach().to(rt.sdtype).contiguous().clone()
        dLdL = torch.zeros((max(rt.S, 1), rt.G), dtype=torch.float64, device=lam.device)
        for s0 in reversed(range(0, steps, K)):
            s1 = min(s0 + K, steps)
            if ctx.last is not None and ctx.last[0] == s0:
                rec = ctx.last[1]
                ctx.last = None
            else:
                U = ctx.ckpts[s0].clone()
                Ub = torch.empty_like(U)
                rec = []
                for _ in range(s0, s1):
                    if rt.S:
                        rt.rt_inject(U, L)
                    UD = rt.rt_gradient(U)
                    Uu = torch.empty_like(U)
                    rt.rt_transport(UD, U_out=Ub, U_unguarded=Uu)
                    U, Ub = Ub, U
                    rec.append((UD, Uu))
            for UD, Uu in reversed(rec):
                rt.rt_adjoint(None, L, lam, lam=lam, UD=UD, U_unguarded=Uu,
                              dL_dL=dLdL if rt.S else None)
            del rec
        ctx.last = None
        gL = dLdL[:rt.S] if rt.S else None
        return gL, lam, None, None, None, None


def rollout(rt, L, U0, steps: int, ckpt_every: int = 5):
    """Differentiable final state after `steps` RT steps (see RTRollout)."""
    keep = torch.is_grad_enabled() and (L.requires_grad or U0.requires_grad)
    return RTRollout.apply(L, U0, rt, steps, ckpt_every, keep)
