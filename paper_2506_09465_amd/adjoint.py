"""Differentiable steady state: a torch.autograd.Function whose forward is the
library's CRN steady solve and whose backward is its adjoint (iugkp_adjoint).

    T = steady_temperature(walls, source, problem, **solver_options)

walls: the wall temperatures, one per wall (2D: left, right, bottom, top; 1D:
left, right), each applied to all faces of its wall; source: the volumetric
heat source per cell (n_cells).  Both are float64 tensors; T is the steady
temperature per cell.  The gradient of any scalar built from T flows back to
walls and source through the adjoint (exact transpose of the common-random-
number map, so it agrees with finite differences of the same forward solve).
"""
from __future__ import annotations

import copy

import torch

from . import _lib as L
from .solver import Solver


def _wall_slices(problem):
    nx, ny = int(problem.nx), int(problem.ny)
    if int(problem.dim) == 1:
        return [slice(0, 1), slice(1, 2)]
    return [slice(0, ny), slice(ny, 2 * ny), slice(2 * ny, 2 * ny + nx),
            slice(2 * ny + nx, 2 * ny + 2 * nx)]


class SteadyState(torch.autograd.Function):
    @staticmethod
    def forward(ctx, walls, source, problem, opts):
        sl = _wall_slices(problem)
        if walls.numel() != len(sl):
            raise ValueError(f"walls needs {len(sl)} values")
        nb = sl[-1].stop
        wall_T = torch.empty(nb, dtype=torch.float64, device=walls.device)
        for i, s in enumerate(sl):
            wall_T[s] = walls[i].to(torch.float64)
        w = copy.copy(problem)
        w.wall_T = wall_T.detach()
        w.source = source.detach().to(torch.float64).contiguous()
        o = dict(opts)
        o["rng_mode"] = L.RNG_CRN
        o.setdefault("tally_faces", L.FACES_OFF)
        adj = {k: o.pop(k) for k in ("adjoint_max_iters", "adjoint_tol") if k in o}
        solver = Solver(w, device=walls.device, **o)
        rc, T, _, _, st = solver.solve()
        ctx.solver = solver
        ctx.slices = sl
        ctx.adj = adj
        ctx.stats = st
        return T

    @staticmethod
    def backward(ctx, grad_T):
        rc, gw, gs, its = ctx.solver.adjoint(grad_T.contiguous(),
                                             max_iters=ctx.adj.get("adjoint_max_iters", 200),
                                             tol=ctx.adj.get("adjoint_tol", 1e-10))
        g4 = torch.stack([gw[s].sum() for s in ctx.slices])
        return g4, gs, None, None


def steady_temperature(walls: torch.Tensor, source: torch.Tensor, problem, **opts) -> torch.Tensor:
    """Steady temperature of `problem` with the given wall temperatures and
    source; differentiable with respect to both.  opts: Solver options plus
    adjoint_max_iters / adjoint_tol for the backward pass."""
    return SteadyState.apply(walls, source, problem, opts)
