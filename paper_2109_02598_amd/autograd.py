"""torch.autograd.Function over the Gray-Scott spectral rollout.

forward:  (u0, v0, coef) -> (u_T, v_T) after `nsteps` semi-implicit
          spectral steps on the GPU (checkpoints every K steps);
backward: the library's hand-written reverse mode (exact transpose of the
          discrete step) gives dJ/du0, dJ/dv0 and dJ/d(Du, Dv, F, k).

Marshalling only: both directions run in the HIP kernels of libspecstep.
"""
from __future__ import annotations

import torch

from . import specstep


class GrayScottRollout(torch.autograd.Function):
    """Apply with ``GrayScottRollout.apply(u0, v0, coef, grid, nsteps, K)``.

    ``grid`` is a specstep.Grid created for the gray_scott model; ``coef``
    a 1-D float64 tensor (Du, Dv, F, k).  The grid holds the forward state
    between forward and backward, so one grid serves one rollout at a time.
    """

    @staticmethod
    def forward(ctx, u0, v0, coef, grid, nsteps, K):
        c = [float(x) for x in coef.detach().cpu().tolist()]
        grid.set_model("gray_scott", c, grid.dt)
        if getattr(grid, "adj_cfg", None) != (int(nsteps), int(K)):
            grid.bind_adjoint(nsteps, K)
        grid.set_field(0, u0.detach())
        grid.set_field(1, v0.detach())
        grid.step_checkpointed()
        uT = grid.get_field(0)
        vT = grid.get_field(1)
        ctx.grid = grid
        ctx.coef_meta = (coef.dtype, coef.device)
        ctx.in_meta = (u0.dtype, u0.device)
        return uT, vT

    @staticmethod
    def backward(ctx, guT, gvT):
        grid = ctx.grid
        if guT is None:
            guT = torch.zeros(grid.shape, dtype=grid.tdtype, device=grid.device)
        if gvT is None:
            gvT = torch.zeros(grid.shape, dtype=grid.tdtype, device=grid.device)
        (du0, dv0), dc = grid.adjoint([guT, gvT])
        dt, dev = ctx.in_meta
        cdt, cdev = ctx.coef_meta
        return (du0.to(dtype=dt, device=dev), dv0.to(dtype=dt, device=dev),
                torch.tensor(dc, dtype=cdt, device=cdev), None, None, None)


def gray_scott_rollout(u0, v0, coef, grid, nsteps, K=20):
    return GrayScottRollout.apply(u0, v0, coef, grid, nsteps, K)
