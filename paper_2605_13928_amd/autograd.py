"""KL(P||Q) as a torch.autograd.Function with hand-written HIP backward.

C = KLDivergence.apply(Y, val, P) differentiates with respect to the 2-D
embedding Y and the stored values `val` of the CSR matrix P (whose pattern
must be symmetric, with tpos).  Forward: tsne_kl_forward (an all-pairs Z
pass plus the sparse sums).  Backward: tsne_kl_backward, which recomputes
the Student-t weights tile by tile (Q is never stored) and returns
gC * dC/dY and gC * dC/dp.  Double backward is not supported.
"""
from __future__ import annotations

import torch

from . import api


class KLDivergence(torch.autograd.Function):
    @staticmethod
    def forward(ctx, Y, val, P):
        Y = Y.contiguous()
        val = val.contiguous()
        C, Z = api.kl_forward(Y, val, P)
        ctx.save_for_backward(Y, val)
        ctx.P = P
        return C

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, gC):
        Y, val = ctx.saved_tensors
        dY, dP = api.kl_backward(Y, val, ctx.P, gC, want_dP=ctx.needs_input_grad[1])
        return (dY if ctx.needs_input_grad[0] else None), dP, None


def kl_divergence(Y: torch.Tensor, val: torch.Tensor, P: api.SparseP) -> torch.Tensor:
    return KLDivergence.apply(Y, val, P)
