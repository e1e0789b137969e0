"""Many independent scenes stepped together: one launch per phase for all of them.

``BatchedParticleSet`` holds the flattened particle arrays of every scene
(scene k owns particles [p_offset_k, p_offset_k + n_k)) and their grids laid
end to end, and runs the batched entry points of the library:

    polypic_batch_sort -> polypic_batch_p2g -> polypic_batch_grid_update
                       -> polypic_batch_g2p (+ advection)

A step can be captured once as a HIP graph (``capture``) and replayed
(``replay``): the positions ping-pong between two buffers, so two graphs are
captured, one per direction.  The coefficients are updated in place (G2P reads
none), as in ``ParticleSet``.  Capture records kernels only (the
library clears grids with a kernel, never with a memset node).
"""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from . import ops


class BatchedParticleSet:
    def __init__(self, grids: Sequence, counts: Sequence[int], n_modes: int, x: torch.Tensor,
                 coeff: torch.Tensor, mass: Optional[torch.Tensor] = None,
                 uniform_mass: float = 1.0, dt: float = 1e-4,
                 gravity: Sequence[float] = (0.0, -9.8, 0.0), bc_layers: int = 1,
                 device: str = "cuda"):
        if n_modes not in ops.ALLOWED_N_MODES:
            raise ValueError(f"n_modes must be one of {ops.ALLOWED_N_MODES}")
        self.batch = ops.Batch(list(zip(grids, counts)), device=device)
        P, N = self.batch.P, self.batch.N
        if x.shape != (3, P) or coeff.shape != (3, n_modes, P):
            raise ValueError(f"x must be (3, {P}) and coeff (3, {n_modes}, {P})")
        f32 = dict(dtype=torch.float32, device=device)
        self.n_modes = n_modes
        self.dt = float(dt)
        self.gravity = tuple(float(g) for g in gravity)
        self.bc_layers = int(bc_layers)
        self.uniform_mass = float(uniform_mass)
        self.x = x.contiguous()
        self.coeff = coeff.contiguous()
        self.mass = None if mass is None else mass.contiguous()
        self.x_next = torch.empty_like(self.x)
        self.coeff_next = self.coeff  # G2P reads no coefficients: in place
        self.mass_next = None if mass is None else torch.empty_like(self.mass)
        self.grid_mass = torch.empty(N, **f32)
        self.grid_mom = torch.empty(3 * N, **f32)
        self.grid_vel = torch.empty(3 * N, **f32)
        self.keys = torch.empty(P, dtype=torch.int32, device=device)
        self.perm = torch.empty(P, dtype=torch.int32, device=device)
        self.sort_ws = torch.empty(max(1, ops.polypic_batch_sort_workspace_bytes(self.batch)),
                                   dtype=torch.uint8, device=device)
        self.status = torch.zeros(1, dtype=torch.int32, device=device)
        self.graphs = None
        self.phase = 0

    @property
    def P(self) -> int:
        return self.batch.P

    def scene_slice(self, k: int) -> slice:
        return slice(self.batch.p_offsets[k], self.batch.p_offsets[k + 1])

    def node_slice(self, k: int) -> slice:
        return slice(self.batch.node_offsets[k], self.batch.node_offsets[k + 1])

    # ---- phases
    def sort(self):
        ops.polypic_batch_sort(self.batch, self.x, self.keys, self.perm, self.sort_ws, self.status)

    def p2g(self, use_perm: bool = True):
        ops.polypic_batch_p2g(self.batch, self.n_modes, self.x, self.coeff, self.grid_mass,
                              self.grid_mom, mass=self.mass, uniform_mass=self.uniform_mass,
                              perm=self.perm if use_perm else None, status_dev=self.status)

    def grid_update(self):
        ops.polypic_batch_grid_update(self.batch, self.dt, self.gravity, self.bc_layers,
                                      self.grid_mass, self.grid_mom, self.grid_vel)

    def g2p(self, use_perm: bool = True):
        ops.polypic_batch_g2p(self.batch, self.n_modes, self.dt, self.grid_vel, self.x,
                              self.coeff_next, perm=self.perm if use_perm else None,
                              x_out=self.x_next, mass_in=self.mass, mass_out=self.mass_next,
                              status_dev=self.status)

    def swap(self):
        self.x, self.x_next = self.x_next, self.x
        if self.mass is not None:
            self.mass, self.mass_next = self.mass_next, self.mass

    def step(self):
        """One eager step for every scene (outputs come out in each scene's cell order)."""
        self.sort()
        self.p2g()
        self.grid_update()
        self.g2p()
        self.swap()
        self.phase ^= 1

    def autotune(self):
        """Sort, then let the library time its batched P2G configurations (synchronises)."""
        self.sort()
        return ops.polypic_batch_autotune(self.batch, self.n_modes, self.x, self.coeff,
                                          self.grid_mass, self.grid_mom, mass=self.mass,
                                          uniform_mass=self.uniform_mass, perm=self.perm)

    # ---- graph capture
    def capture(self):
        """Capture one step in each buffer direction as a HIP graph (no work is run)."""
        torch.cuda.synchronize()
        graphs = []
        for _ in range(2):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                self.sort()
                self.p2g()
                self.grid_update()
                self.g2p()
            graphs.append(g)
            self.swap()       # the second graph reads what the first one writes
        # two swaps: the buffers are back where they started, and graphs[0]
        # runs in the current direction
        self.graphs = graphs
        self.phase = 0

    def replay(self):
        """One step through the captured graph of the current direction."""
        if self.graphs is None:
            raise RuntimeError("capture() first")
        self.graphs[self.phase].replay()
        self.swap()
        self.phase ^= 1

    def status_flags(self) -> int:
        return int(self.status.item())
