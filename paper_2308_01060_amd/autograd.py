"""Differentiable multi-step transfers: ``PolyPICSteps`` (a torch.autograd.Function).

Forward: S steps of sort -> P2G -> grid update -> G2P + advection through the
library, keeping one checkpoint (x_s, c_s) per step.  Backward: for
s = S-1 .. 0 the step's sort, P2G and grid update are recomputed from the
checkpoint (the stencil weights are never stored), then

    polypic_g2p_backward -> polypic_grid_update_backward -> polypic_p2g_backward

carry dL/d(x_{s+1}, c_{s+1}) to dL/d(x_s, c_s).  Each step's outputs come out
in its sort order; the function returns (x_S, c_S) in the caller's particle
order and its gradients in that order too.
"""
from __future__ import annotations

from typing import Sequence

import torch

from . import ops


class _Buffers:
    """Device work buffers shared by the forward and backward passes."""

    def __init__(self, grid, P: int, n_modes: int, device):
        f32 = dict(dtype=torch.float32, device=device)
        N = ops.n_nodes(grid)
        self.gm = torch.empty(N, **f32)
        self.gp = torch.empty(3 * N, **f32)
        self.gv = torch.empty(3 * N, **f32)
        self.gvb = torch.empty(3 * N, **f32)
        self.gmb = torch.empty(N, **f32)
        self.gpb = torch.empty(3 * N, **f32)
        self.keys = torch.empty(P, dtype=torch.int32, device=device)
        self.perm = torch.empty(P, dtype=torch.int32, device=device)
        self.sort_ws = torch.empty(max(1, ops.polypic_sort_workspace_bytes(grid, P)),
                                   dtype=torch.uint8, device=device)
        self.p2g_ws = torch.empty(max(1, ops.polypic_p2g_workspace_bytes(grid, P)),
                                  dtype=torch.uint8, device=device)
        self.status = torch.zeros(1, dtype=torch.int32, device=device)


def _forward_grid(grid, n_modes, dt, gravity, bc_layers, uniform_mass, x, c, B: _Buffers):
    """sort + P2G + grid update for the step whose inputs are (x, c)."""
    ops.polypic_sort(grid, x, B.keys, B.perm, B.sort_ws, B.status)
    ops.polypic_p2g(grid, n_modes, x, c, B.gm, B.gp, uniform_mass=uniform_mass, perm=B.perm,
                    keys_sorted=B.keys, ws=B.p2g_ws, status_dev=B.status)
    ops.polypic_grid_update(grid, dt, gravity, bc_layers, B.gm, B.gp, B.gv)


class PolyPICSteps(torch.autograd.Function):
    """(x0 [3, P], c0 [3, n_modes, P]) -> (x_S, c_S) after n_steps transfer steps."""

    @staticmethod
    def forward(ctx, x0, c0, grid, n_modes: int, n_steps: int, dt: float,
                gravity: Sequence[float], bc_layers: int, uniform_mass: float = 1.0):
        P = x0.shape[-1]
        dev = x0.device
        B = _Buffers(grid, P, n_modes, dev)
        x = x0.detach().contiguous().reshape(3, P)
        c = c0.detach().contiguous().reshape(3, n_modes, P)
        order = torch.arange(P, dtype=torch.int64, device=dev)
        checkpoints = []
        for _ in range(n_steps):
            checkpoints.append((x, c))
            _forward_grid(grid, n_modes, dt, gravity, bc_layers, uniform_mass, x, c, B)
            x_next = torch.empty_like(x)
            c_next = torch.empty_like(c)
            ops.polypic_g2p(grid, n_modes, dt, B.gv, x, c_next, perm=B.perm, x_out=x_next,
                            status_dev=B.status)
            order = order[B.perm.long()]
            x, c = x_next, c_next
        ctx.grid = grid
        ctx.params = (n_modes, n_steps, float(dt), tuple(float(g) for g in gravity),
                      int(bc_layers), float(uniform_mass))
        ctx.checkpoints = checkpoints
        ctx.buffers = B
        ctx.save_for_backward(order)
        x_out = torch.empty_like(x)
        c_out = torch.empty_like(c)
        x_out[:, order] = x
        c_out[:, :, order] = c
        return x_out, c_out

    @staticmethod
    def backward(ctx, gx_out, gc_out):
        (order,) = ctx.saved_tensors
        n_modes, n_steps, dt, gravity, bc_layers, uniform_mass = ctx.params
        grid, B = ctx.grid, ctx.buffers
        P = order.numel()
        if gx_out is None:
            gx_out = torch.zeros(3, P, dtype=torch.float32, device=order.device)
        if gc_out is None:
            gc_out = torch.zeros(3, n_modes, P, dtype=torch.float32, device=order.device)
        # to the slot order of the last step's outputs
        gx = gx_out.float()[:, order].contiguous()
        gc = gc_out.float()[:, :, order].contiguous()
        for s in range(n_steps - 1, -1, -1):
            x, c = ctx.checkpoints[s]
            _forward_grid(grid, n_modes, dt, gravity, bc_layers, uniform_mass, x, c, B)
            gx_in = torch.zeros_like(gx)
            gc_in = torch.empty_like(gc)
            ops.polypic_g2p_backward(grid, n_modes, dt, B.gv, x, gc, B.gvb, gx_in, perm=B.perm,
                                     x_out_grad=gx, status_dev=B.status)
            ops.polypic_grid_update_backward(grid, dt, gravity, bc_layers, B.gm, B.gp, B.gvb,
                                             B.gmb, B.gpb)
            # the P2G adjoint is a gather: particle order keeps its particle streams coalesced
            ops.polypic_p2g_backward(grid, n_modes, x, c, B.gmb, B.gpb, gc_in, gx_in,
                                     uniform_mass=uniform_mass, status_dev=B.status)
            gx, gc = gx_in, gc_in
        ctx.checkpoints = None
        return gx, gc, None, None, None, None, None, None, None


def polypic_steps(x0, c0, grid, n_modes: int, n_steps: int, dt: float,
                  gravity: Sequence[float] = (0.0, -9.8, 0.0), bc_layers: int = 1,
                  uniform_mass: float = 1.0):
    """Differentiable n_steps of transfers; returns (x_S, c_S) in the input particle order."""
    return PolyPICSteps.apply(x0, c0, grid, n_modes, n_steps, dt, gravity, bc_layers,
                              uniform_mass)
