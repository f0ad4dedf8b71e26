"""Reverse-mode differentiation through the library's kernels.

`deriv(cells, y, lnk)` returns f(y; k = exp(lnk)) for every cell of a batch,
as a torch tensor that autograd can differentiate with respect to y and the
log rate constants: the backward pass is one launch of the library's VJP
kernel (mcc_calc_vjp): dL/dy = J^T g and dL/d ln k_j = r_j sum_i nu_ij g_i for
the incoming gradient g = dL/df.  The exp of the parameter is torch
arithmetic on the parameter tensor; f and both products run in the library.

`solve_step(cells, y0, lnk, dt)` is one outer step of the BDF solver,
y(dt) for every cell, differentiable with respect to y0 and ln k: the
forward pass records each cell's step tape (mcc_solve_step_taped) and the
backward pass is the discrete adjoint of that step sequence
(mcc_adjoint_step), both in the library.
"""
from __future__ import annotations

import torch

from . import mcchem


def _check_forward(status: torch.Tensor) -> None:
    """A cell that did not reach the end of its outer step (too much work, a
    convergence, error-test or non-finite failure) has no derivative of the
    map being differentiated: refuse it rather than return a state short of dt."""
    if status.numel() and int((status != mcchem.CELL_OK).sum()) > 0:
        bad = torch.unique(status[status != mcchem.CELL_OK]).tolist()
        raise mcchem.MccError("forward step failed for some cells (status " +
                              ", ".join(mcchem.CELL_STATUS.get(int(s), str(s)) for s in bad) + ")")


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


class _SolveStep(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y0, lnk, cells, dt, opts, stride):
        k = torch.exp(lnk).contiguous()
        cells.set_rate_constants(k)
        y0 = y0.contiguous()
        while True:
            y = y0.clone()
            tape = torch.empty((cells.n_cells, stride), dtype=torch.float64, device=y0.device)
            tape_len = torch.empty(cells.n_cells, dtype=torch.int64, device=y0.device)
            status, _ = cells.step_taped(y, dt, tape, tape_len, opts)
            if cells.n_cells == 0 or int(tape_len.min()) >= 0:
                break
            stride *= 2  # a tape did not fit: the same step again with room for it
        _check_forward(status)
        ctx.save_for_backward(y0, k, tape, tape_len)
        ctx.cells = cells
        return y

    @staticmethod
    def backward(ctx, g):
        y0, k, tape, tape_len = ctx.saved_tensors
        cells = ctx.cells
        cells.set_rate_constants(k)
        lam = g.contiguous().clone()
        glnk, status = cells.adjoint_step(y0, tape, tape_len, lam)
        if int((status != mcchem.CELL_OK).sum()) > 0:
            raise mcchem.MccError("reverse-mode step failed for some cells: "
                                  f"{torch.unique(status).tolist()}")
        return lam, glnk, None, None, None, None


def solve_step(cells: "mcchem.Cells", y0: torch.Tensor, lnk: torch.Tensor, dt: float,
               opts: "mcchem.SolverOpts | None" = None, tape_stride: int | None = None) -> torch.Tensor:
    """y(dt) [N][ld] from y0 [N][ld] with rate constants exp(lnk) [R][ld].
    tape_stride: doubles of step tape per cell (default room for about 256
    steps; doubled and the step redone when a tape does not fit)."""
    N = cells.mech.n_species
    stride = tape_stride or 4 + 256 * (N + 16)
    return _SolveStep.apply(y0, lnk, cells, dt, opts, stride)


def _tape_bound(stats, n_species: int) -> int:
    """Doubles of step tape the largest cell of an outer step needs (the
    bound of mcc_solve_step_taped: 4 + 8 attempts + n_species steps)."""
    sn = mcchem.stats_numpy(stats)
    attempts = sn["steps"].astype("int64") + sn["rejects"] + sn["newton_fails"]
    return int((4 + 8 * attempts + n_species * sn["steps"].astype("int64")).max()) if len(sn) else 4


class _Integrate(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y0, lnk, cells, dt, n_steps, opts):
        k = torch.exp(lnk).contiguous()
        cells.set_rate_constants(k)
        N = cells.mech.n_species
        y = y0.contiguous().clone()
        checkpoints, stride = [], 4
        stats = None
        for _ in range(n_steps):
            checkpoints.append(y.clone())  # the state each outer step starts from
            status, stats = cells.step(y, dt, opts, stats=stats)
            _check_forward(status)
            stride = max(stride, _tape_bound(stats, N))
        ctx.save_for_backward(k, *checkpoints)
        ctx.cells, ctx.dt, ctx.opts, ctx.stride = cells, dt, opts, stride
        return y

    @staticmethod
    def backward(ctx, g):
        k, *checkpoints = ctx.saved_tensors
        cells = ctx.cells
        cells.set_rate_constants(k)
        C = cells.n_cells
        lam = g.contiguous().clone()
        glnk = torch.zeros((cells.mech.n_reactions, cells.ld), dtype=torch.float64, device=g.device)
        tape = torch.empty((C, ctx.stride), dtype=torch.float64, device=g.device)
        tlen = torch.empty(C, dtype=torch.int64, device=g.device)
        status = torch.empty(C, dtype=torch.int32, device=g.device)
        for y_start in reversed(checkpoints):
            # recompute the outer step's tape from its checkpoint (the solver is
            # deterministic: the same steps as the forward pass), then reverse it
            y = y_start.clone()
            cells.step_taped(y, ctx.dt, tape, tlen, ctx.opts)
            cells.adjoint_step(y_start, tape, tlen, lam, glnk, accumulate=True, status=status)
            if int((status != mcchem.CELL_OK).sum()) > 0:
                raise mcchem.MccError(f"reverse-mode step failed for some cells: {torch.unique(status).tolist()}")
        return lam, glnk, None, None, None, None


def integrate(cells: "mcchem.Cells", y0: torch.Tensor, lnk: torch.Tensor, dt: float, n_steps: int,
              opts: "mcchem.SolverOpts | None" = None) -> torch.Tensor:
    """y after n_steps outer steps of length dt, differentiable with respect
    to y0 [N][ld] and ln k [R][ld].  The forward pass keeps only the state at
    the start of every outer step (checkpoints); the backward pass re-runs
    each outer step from its checkpoint with its step tape and reverses it,
    last step first, accumulating d L / d ln k."""
    return _Integrate.apply(y0, lnk, cells, dt, n_steps, opts)
