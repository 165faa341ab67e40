"""Differentiable mover -> moment gather of one species (Eqs. 1-5, 8).

``move_moments(grid, qom, q, pos, vel, E, B, cell=None)`` returns (J, M): the
particles are moved with (E, B) (Eqs. 4, 5, 8) and their moments J-hat (Eq. 1)
and the 14 stored mass-matrix blocks (Eq. 3) deposited at the new positions
with the same B. Gradients of any loss of J and M flow to the pre-move
positions and velocities and to the grid fields E and B through the
hand-written adjoint (ecsim_moments_backward through the mover). Forward and
backward both run in the library's kernels; the inputs are not modified and
only they are saved.

FP64 form: ``pos`` holds absolute positions. FP32 form: ``pos`` holds the
in-cell offsets and ``cell`` the int32 cell indices; the position gradient is
then taken with respect to the offsets (the library's ECSIM_BWD_OFFSET_GRAD).
"""
from typing import Optional

import torch

from . import ecsim as _E


def _species(prec, qom, q, pos, vel, cell):
    qa, qc = (None, float(q)) if not torch.is_tensor(q) else (q, 0.0)
    return _E.Species(prec, float(qom), pos, vel, cell, qa, qc)


class MoveMoments(torch.autograd.Function):
    @staticmethod
    def forward(ctx, grid, qom, q, pos, vel, E, B, cell):
        prec = _E.F32 if pos.dtype == torch.float32 else _E.F64
        moved = _species(prec, qom, q, pos.detach().clone(), vel.detach().clone(),
                         None if cell is None else cell.clone())
        _E.move(grid, moved, E.detach(), B.detach())
        J = torch.empty((3, grid.nn), dtype=pos.dtype, device=pos.device)
        M = torch.empty((14, 9, grid.nn), dtype=pos.dtype, device=pos.device)
        _E.moments(grid, [moved], B.detach(), J, M)
        ctx.grid, ctx.qom, ctx.q, ctx.prec = grid, qom, q, prec
        ctx.save_for_backward(pos, vel, E, B, cell)
        return J, M

    @staticmethod
    def backward(ctx, gJ, gM):
        pos, vel, E, B, cell = ctx.saved_tensors
        grid = ctx.grid
        sp = _species(ctx.prec, ctx.qom, ctx.q, pos.detach(), vel.detach(), cell)
        gpos = torch.empty_like(pos)
        gvel = torch.empty_like(vel)
        gE = torch.zeros_like(E)
        gB = torch.zeros_like(B)
        zJ = torch.zeros((3, grid.nn), dtype=pos.dtype, device=pos.device) if gJ is None else gJ.contiguous()
        zM = torch.zeros((14, 9, grid.nn), dtype=pos.dtype, device=pos.device) if gM is None else gM.contiguous()
        _E.moments_backward(grid, sp, E.detach(), B.detach(), zJ, zM, gpos, gvel, gE, gB, through_mover=True,
                            offset_grad=ctx.prec == _E.F32)
        return None, None, None, gpos, gvel, gE, gB, None


def move_moments(grid: "_E.Grid", qom: float, q, pos: torch.Tensor, vel: torch.Tensor, E: torch.Tensor,
                 B: torch.Tensor, cell: Optional[torch.Tensor] = None):
    """(J, M) of the moved species; differentiable in pos, vel, E and B. ``q`` is a per-particle
    charge tensor or one charge for all."""
    return MoveMoments.apply(grid, qom, q, pos, vel, E, B, cell)
