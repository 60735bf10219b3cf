"""Differentiation through the BTTB operators: torch.autograd.Functions whose backward
is the hand-written transpose product (and vice versa), so first and second
derivatives both run in the HIP library."""
from __future__ import annotations

import torch

from .operator import Operator


class BTTBFunction(torch.autograd.Function):
    """y = A m for m [..., nz, nx, ny]; the gradient of <g, A m> with respect to m is A^T g."""

    @staticmethod
    def forward(ctx, m: torch.Tensor, op: Operator) -> torch.Tensor:
        ctx.op = op
        return op.matvec(m.contiguous())

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        return BTTBTransposeFunction.apply(g.contiguous(), ctx.op), None


class BTTBTransposeFunction(torch.autograd.Function):
    """z = A^T r for r [..., sx, sy]; its gradient is the forward product."""

    @staticmethod
    def forward(ctx, r: torch.Tensor, op: Operator) -> torch.Tensor:
        ctx.op = op
        return op.rmatvec(r.contiguous())

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        return BTTBFunction.apply(g.contiguous(), ctx.op), None


def forward(m: torch.Tensor, op: Operator) -> torch.Tensor:
    return BTTBFunction.apply(m, op)


def transpose(r: torch.Tensor, op: Operator) -> torch.Tensor:
    return BTTBTransposeFunction.apply(r, op)


class ForwardModel(torch.nn.Module):
    """Module form: predicted data of a batch of models through one operator."""

    def __init__(self, op: Operator):
        super().__init__()
        self.op = op

    def forward(self, m: torch.Tensor) -> torch.Tensor:
        return BTTBFunction.apply(m, self.op)
