"""Differentiable SPC5 product y = A(theta) x for torch.autograd.

theta holds the matrix's nonzeros in SPC5 packed order (the order of
Spc5Matrix.export()); the sparsity pattern (anchors and masks) is fixed.
Backward, both in HIP kernels of libspc5:
  xbar     = A(theta)^T ybar   (spc5_spmv_transpose_values through the
                                matrix's transpose plan: products formed in
                                A's order, summed in A^T's order, no atomics)
  thetabar = ybar[row(v)] * x[col(v)] in packed order (spc5_values_grad)
The forward builds the transpose plan when the matrix has none (once, before
the first backward); the atomic scatter without a plan is never used here.
This module only wires the calls; it computes nothing itself.
"""
from __future__ import annotations

import torch

from .spc5 import Spc5Matrix


class Spc5MatVec(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta: torch.Tensor, x: torch.Tensor, A: Spc5Matrix):
        if not A.has_transpose_plan:
            A.prepare_transpose()
        theta = theta.contiguous()
        x = x.contiguous()
        y = A.spmv_values(theta, x)
        ctx.A = A
        ctx.save_for_backward(theta, x)
        return y

    @staticmethod
    def backward(ctx, ybar: torch.Tensor):
        theta, x = ctx.saved_tensors
        A: Spc5Matrix = ctx.A
        ybar = ybar.contiguous()
        gtheta = gx = None
        if ctx.needs_input_grad[0]:
            gtheta = A.values_grad(ybar, x)
        if ctx.needs_input_grad[1]:
            gx = A.transpose(ybar, values=theta)
        return gtheta, gx, None


def spc5_matvec(A: Spc5Matrix, theta: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    """y = A(theta) x, differentiable in theta and x."""
    return Spc5MatVec.apply(theta, x, A)


class Spc5Linear(torch.nn.Module):
    """A sparse linear map with a fixed SPC5 pattern and trainable values.

    forward(x) = A(theta) x for a vector x of length ncols.
    """

    def __init__(self, A: Spc5Matrix, theta: torch.Tensor, transpose_plan: bool = True):
        super().__init__()
        if transpose_plan:
            A.prepare_transpose()
        self.A = A
        self.theta = torch.nn.Parameter(theta)

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        return spc5_matvec(self.A, self.theta, x)
