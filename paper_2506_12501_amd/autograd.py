"""torch.autograd front end: integrals of one class batch as a function of
the shell centres.  The forward pass calls mdx_eri_batch, the backward pass
mdx_eri_grad_batch with the incoming gradient as the adjoint; the twelve
per-shellset centre derivatives are then summed onto the shells they belong
to (index_add_ over the pair lists).
"""
from __future__ import annotations

import numpy as np
import torch

from . import native


class ERIFunction(torch.autograd.Function):
    """ERIFunction.apply(center, shells, ncentre, bra, ket, cartesian) ->
    integrals [nbra, nab, ncd, nket]; center is a float64 [nshell, 3] device
    tensor that replaces the shell table's centres."""

    @staticmethod
    def forward(ctx, center, shells, ncentre, bra, ket, cartesian=False):
        bra = np.ascontiguousarray(np.asarray(bra, dtype=np.int32).reshape(-1, 2))
        ket = np.ascontiguousarray(np.asarray(ket, dtype=np.int32).reshape(-1, 2))
        sh = shells.with_center(center.detach())
        out = native.eri(sh, ncentre, bra, ket, cartesian=cartesian)
        ctx.save_for_backward(center)
        ctx.args = (shells, ncentre, bra, ket, cartesian)
        return out

    @staticmethod
    def backward(ctx, gout):
        (center,) = ctx.saved_tensors
        shells, ncentre, bra, ket, cartesian = ctx.args
        sh = shells.with_center(center.detach())
        g = native.eri_grad(sh, ncentre, bra, ket, gout.contiguous() if gout.dim() != 4 else gout,
                            cartesian=cartesian)   # [nbra, 12, nket]
        gc = torch.zeros(center.shape[0], 3, dtype=torch.float64, device=center.device)
        dev = center.device
        # slots (A, B) belong to the bra pair, (C, D) to the ket pair
        for X, (lst, col, axis) in enumerate(((bra, 0, 2), (bra, 1, 2), (ket, 0, 0), (ket, 1, 0))):
            idx = lst[:, col]
            if idx[0] < 0:   # absent function of a 3-/2-centre side
                continue
            part = g[:, 3 * X:3 * X + 3, :].sum(dim=axis)          # [nbra, 3] or [3, nket]
            if axis == 0:
                part = part.transpose(0, 1)
            gc.index_add_(0, torch.as_tensor(idx, dtype=torch.int64, device=dev), part)
        return gc.reshape(center.shape), None, None, None, None, None


def eri(center, shells, ncentre, bra, ket, cartesian=False):
    return ERIFunction.apply(center, shells, ncentre, bra, ket, cartesian)
