"""Differentiable multi-step transfers: ``PolyPICSteps`` (a torch.autograd.Function).

Forward: S steps run as the library steps a ParticleSet -- the sort (the exact
re-sort from the previous step's keys after the first), the grid update, and
G2P + advection fused with the next step's P2G (``polypic_g2p2g``; the first
step's P2G and the last step's G2P are separate calls).  Per step it keeps a
checkpoint: the particle state (x_s, c_s), the sort permutation and the grid
fields (mass, momentum, velocity) -- 81 MB per step at 132^3 nodes and 4.19 M
particles, beside the 1.4 GB of particle state.  The stencil weights are never
stored.  Backward, for s = S-1 .. 0:

    polypic_g2p_backward -> polypic_grid_update_backward -> polypic_p2g_backward

carry dL/d(x_{s+1}, c_{s+1}) to dL/d(x_s, c_s), each kernel recomputing the
weights from x_s.  Each step's outputs come out in its sort order; the function
returns (x_S, c_S) in the caller's particle order and its gradients in that
order too.
"""
from __future__ import annotations

from typing import Sequence

import torch

from . import _lib, ops


def _raise_on_flags(status: torch.Tensor, where: str) -> None:
    """Read the device flag word (one synchronisation) and raise if any flag is set: an
    out-of-range particle (skipped by every kernel), keys out of order in a re-sort, or a
    re-sort that gave up waiting, each of which would otherwise leave wrong outputs or zero
    gradients without an error."""
    flags = int(status.item())
    if flags:
        names = [n for bit, n in ((_lib.POLYPIC_FLAG_RANGE, "a particle stencil left the grid"),
                                  (_lib.POLYPIC_FLAG_ORDER, "re-sort keys out of order"),
                                  (_lib.POLYPIC_FLAG_STALL, "re-sort stalled")) if flags & bit]
        raise _lib.PolyPICError(_lib.POLYPIC_EINVAL if flags & _lib.POLYPIC_FLAG_RANGE
                                else _lib.POLYPIC_EDEVICE,
                                f"{where}: device flags {flags} ({'; '.join(names)})")


class _Buffers:
    """Device work buffers shared by the forward and backward passes."""

    def __init__(self, grid, P: int, n_modes: int, device):
        f32 = dict(dtype=torch.float32, device=device)
        N = ops.n_nodes(grid)
        self.N = N
        self.gvb = torch.empty(3 * N, **f32)
        self.gmb = torch.empty(N, **f32)
        self.gpb = torch.empty(3 * N, **f32)
        self.keys = [torch.empty(P, dtype=torch.int32, device=device) for _ in range(2)]
        self.sort_ws = torch.empty(max(1, ops.polypic_sort_workspace_bytes(grid, P)),
                                   dtype=torch.uint8, device=device)
        self.resort_ws = torch.empty(max(1, ops.polypic_sort_update_workspace_bytes(grid, P)),
                                     dtype=torch.uint8, device=device)
        self.p2g_ws = torch.empty(max(1, ops.polypic_p2g_workspace_bytes(grid, P)),
                                  dtype=torch.uint8, device=device)
        self.status = torch.zeros(1, dtype=torch.int32, device=device)


class PolyPICSteps(torch.autograd.Function):
    """(x0 [3, P], c0 [3, n_modes, P]) -> (x_S, c_S) after n_steps transfer steps."""

    @staticmethod
    def forward(ctx, x0, c0, grid, n_modes: int, n_steps: int, dt: float,
                gravity: Sequence[float], bc_layers: int, uniform_mass: float = 1.0,
                check_status: bool = True):
        P = x0.shape[-1]
        dev = x0.device
        B = _Buffers(grid, P, n_modes, dev)
        N = B.N
        f32 = dict(dtype=torch.float32, device=dev)
        x = x0.detach().contiguous().reshape(3, P)
        c = c0.detach().contiguous().reshape(3, n_modes, P)
        order = torch.arange(P, dtype=torch.int32, device=dev)  # particle of each slot
        checkpoints = []
        gm = torch.empty(N, **f32)
        gp = torch.empty(3 * N, **f32)
        for s in range(n_steps):
            keys, keys_prev = B.keys[s % 2], B.keys[(s + 1) % 2]
            perm = torch.empty(P, dtype=torch.int32, device=dev)
            if s == 0:
                ops.polypic_sort(grid, x, keys, perm, B.sort_ws, B.status)
                ops.polypic_p2g(grid, n_modes, x, c, gm, gp, uniform_mass=uniform_mass,
                                perm=perm, keys_sorted=keys, ws=B.p2g_ws, status_dev=B.status)
            else:
                # slot i of x was written from the previous sort's slot i: sorted under
                # keys_prev[i]
                ops.polypic_sort_update(grid, x, keys_prev, keys, perm, B.resort_ws, B.status)
            gv = torch.empty(3 * N, **f32)
            ops.polypic_grid_update(grid, dt, gravity, bc_layers, gm, gp, gv)
            checkpoints.append((x, c, perm, gm, gp, gv))
            x_next = torch.empty_like(x)
            c_next = torch.empty_like(c)
            if s + 1 < n_steps:
                gm, gp = torch.empty(N, **f32), torch.empty(3 * N, **f32)
                ops.polypic_g2p2g(grid, n_modes, dt, gv, x, x_next, c_next, gm, gp, perm=perm,
                                  uniform_mass=uniform_mass, status_dev=B.status)
            else:
                ops.polypic_g2p(grid, n_modes, dt, gv, x, c_next, perm=perm, x_out=x_next,
                                status_dev=B.status)
            new_order = torch.empty_like(order)
            ops.polypic_gather_rows(order, new_order, perm)  # slot i now holds order[perm[i]]
            order = new_order
            x, c = x_next, c_next
        if check_status:
            _raise_on_flags(B.status, "PolyPICSteps forward")
        ctx.grid = grid
        ctx.check_status = bool(check_status)
        ctx.params = (n_modes, n_steps, float(dt), tuple(float(g) for g in gravity),
                      int(bc_layers), float(uniform_mass))
        ctx.checkpoints = checkpoints
        ctx.buffers = B
        ctx.save_for_backward(order)
        # back to the caller's particle order: out[order[i]] = state[i]
        x_out = torch.empty_like(x)
        c_out = torch.empty_like(c)
        ops.polypic_scatter_rows(x, x_out, order)
        ops.polypic_scatter_rows(c, c_out, order)
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
        gx = torch.empty(3, P, dtype=torch.float32, device=order.device)
        gc = torch.empty(3, n_modes, P, dtype=torch.float32, device=order.device)
        ops.polypic_gather_rows(gx_out.float().contiguous().reshape(3, P), gx, order)
        ops.polypic_gather_rows(gc_out.float().contiguous().reshape(3, n_modes, P), gc, order)
        for s in range(n_steps - 1, -1, -1):
            x, c, perm, gm, gp, gv = ctx.checkpoints[s]
            gx_in = torch.zeros_like(gx)
            gc_in = torch.empty_like(gc)
            ops.polypic_g2p_backward(grid, n_modes, dt, gv, x, gc, B.gvb, gx_in, perm=perm,
                                     x_out_grad=gx, status_dev=B.status)
            ops.polypic_grid_update_backward(grid, dt, gravity, bc_layers, gm, gp, B.gvb,
                                             B.gmb, B.gpb)
            # the P2G adjoint is a gather: particle order keeps its particle streams coalesced
            ops.polypic_p2g_backward(grid, n_modes, x, c, B.gmb, B.gpb, gc_in, gx_in,
                                     uniform_mass=uniform_mass, status_dev=B.status)
            gx, gc = gx_in, gc_in
            ctx.checkpoints[s] = None  # released as soon as its step is done
        ctx.checkpoints = None
        if ctx.check_status:
            _raise_on_flags(B.status, "PolyPICSteps backward")
        return gx, gc, None, None, None, None, None, None, None, None


def polypic_steps(x0, c0, grid, n_modes: int, n_steps: int, dt: float,
                  gravity: Sequence[float] = (0.0, -9.8, 0.0), bc_layers: int = 1,
                  uniform_mass: float = 1.0, check_status: bool = True):
    """Differentiable n_steps of transfers; returns (x_S, c_S) in the input particle order.

    With check_status (the default) the forward and the backward each read the device flag
    word once at their end and raise PolyPICError if a kernel flagged a particle out of
    range or a failed re-sort (one synchronisation each)."""
    return PolyPICSteps.apply(x0, c0, grid, n_modes, n_steps, dt, gravity, bc_layers,
                              uniform_mass, check_status)
