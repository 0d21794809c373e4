"""Differentiable matrix profile: torch.autograd.Function over the batched
self-join (forward) and the library's backward kernel (dL/dT through each
row's argmin pair, index held fixed)."""

from __future__ import annotations

import torch

from ._binding import BatchPlan


class MatrixProfileFn(torch.autograd.Function):
    """P, I = MatrixProfileFn.apply(T, plan) for T of shape [B, n] (equal
    lengths) or the concatenated 1-D layout of `plan`.  P is differentiable;
    I is marked non-differentiable."""

    @staticmethod
    def forward(ctx, T, plan: BatchPlan):
        Tc = T.reshape(-1).contiguous()
        P, I = plan.run(Tc)
        ctx.plan = plan
        ctx.shape = T.shape
        ctx.forward_id = plan.forward_count
        ctx.save_for_backward(Tc, I, P)
        ctx.mark_non_differentiable(I)
        if T.dim() == 2:
            B = T.shape[0]
            return P.view(B, -1), I.view(B, -1)
        return P, I

    @staticmethod
    def backward(ctx, gP, gI):
        # (autograd refuses saved tensors modified in place, so T is the
        # forward's; the plan's workspace still holds this forward's window
        # statistics while no other forward has run on it)
        Tc, I, P = ctx.saved_tensors
        gP = torch.nan_to_num(gP.reshape(-1), nan=0.0, posinf=0.0, neginf=0.0)
        plan = ctx.plan
        if plan.reuses_forward and plan.forward_count == ctx.forward_id:
            gT = plan.backward_after_forward(Tc, I, P, gP)
        else:
            gT = plan.backward(Tc, I, gP)
        return gT.view(ctx.shape), None


def matrix_profile(T: torch.Tensor, m: int, ez: int, plan: BatchPlan | None = None, **plan_kw):
    """Differentiable profile of a [B, n] batch of equal-length series."""
    if T.dim() != 2:
        raise ValueError("T must be [B, n]")
    B, n = T.shape
    if plan is None:
        plan = BatchPlan([n] * B, [m] * B, [ez] * B, dtype=T.dtype, device=T.device, **plan_kw)
    return MatrixProfileFn.apply(T, plan)


def abjoin_profile(A: torch.Tensor, B: torch.Tensor, m: int, plan=None, **plan_kw):
    """Differentiable AB-join: (P_ab, I_ab, P_ba, I_ba) with gradients
    flowing to A and B through both profiles (indices held fixed)."""
    from ._binding import ABJoinPlan
    if A.dim() != 1 or B.dim() != 1:
        raise ValueError("A and B must be 1-D")
    if plan is None:
        plan = ABJoinPlan(A.numel(), B.numel(), m, dtype=A.dtype, device=A.device, **plan_kw)
    T = torch.cat([A, B])          # the plan's layout: A then B
    P, I = MatrixProfileFn.apply(T, plan)
    lA = A.numel() - m + 1
    return P[:lA], I[:lA], P[lA:], I[lA:]
