"""The reconstruction xhat as a torch.autograd.Function.

forward:  xhat_x = sum_r prod_n C(n)[i_n, r] for every element x of a plan, in input order
          (Eq. (1) through Eq. (12)), C(n) = A(n) B(n) recomputed into scratch.
backward: for dL/dxhat = delta, the gradients of Eq. (10) and Eq. (11) without the regulariser:
          dA(n)[i] = sum_{x: i_n = i} delta_x B(n) w(n)_x,  dB(n) = sum_x delta_x A(n)[i_n]^T w(n)_x,
          computed by the library's segment kernels.  C is recomputed, not kept from forward.
Both directions run in the HIP library (ft_forward / ft_grad); this module only marshals tensors.
"""
from __future__ import annotations

import torch

from . import api


def _params(plan, A, B, storage):
    p = api.Params([a.detach() for a in A], [b.detach() for b in B], device=A[0].device, storage=storage)
    api.refresh(plan, p)
    return p


class Reconstruction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, storage, *params):
        N = plan.order
        A, B = params[:N], params[N:]
        if len(B) != N:
            raise ValueError("expected A(0..N-1) then B(0..N-1)")
        p = _params(plan, A, B, storage)
        out = api.forward(plan, p)
        ctx.plan = plan
        ctx.storage = storage
        ctx.save_for_backward(*A, *B)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        plan = ctx.plan
        N = plan.order
        saved = ctx.saved_tensors
        p = _params(plan, saved[:N], saved[N:], ctx.storage)
        gA, gB = api.grad(plan, p, grad_out.contiguous())
        return (None, None, *gA, *gB)


def reconstruct(plan, A, B, storage="f32"):
    """xhat (input order) as a differentiable function of the lists A and B; the plan needs with_perm=True.

    storage "bf16" evaluates forward and backward on BF16 copies of A, B, C with FP32 accumulation;
    the gradients are FP32 tensors for the FP32 leaves A, B."""
    return Reconstruction.apply(plan, storage, *A, *B)
