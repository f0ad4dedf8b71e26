"""Reverse-mode differentiation of f through the library's kernels.

`deriv(cells, y, lnk)` returns f(y; k = exp(lnk)) for every cell of a batch,
as a torch tensor that autograd can differentiate with respect to y and the
log rate constants: the backward pass is one launch of the library's VJP
kernel (mcc_calc_vjp): dL/dy = J^T g and dL/d ln k_j = r_j sum_i nu_ij g_i for
the incoming gradient g = dL/df.  The exp of the parameter is torch
arithmetic on the parameter tensor; f and both products run in the library.
"""
from __future__ import annotations

import torch

from . import mcchem


class _Deriv(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y, lnk, cells):
        k = torch.exp(lnk).contiguous()
        cells.set_rate_constants(k)
        f = cells.deriv(y.contiguous())
        ctx.save_for_backward(y, k)
        ctx.cells = cells
        return f

    @staticmethod
    def backward(ctx, g):
        y, k = ctx.saved_tensors
        cells = ctx.cells
        cells.set_rate_constants(k)  # the batch may have been rebound since forward
        gy, glnk = cells.vjp(y.contiguous(), g.contiguous(), want_gy=ctx.needs_input_grad[0],
                             want_glnk=ctx.needs_input_grad[1])
        return gy, glnk, None


def deriv(cells: "mcchem.Cells", y: torch.Tensor, lnk: torch.Tensor) -> torch.Tensor:
    """f [N][ld] at y [N][ld] with rate constants exp(lnk) [R][ld]."""
    return _Deriv.apply(y, lnk, cells)
