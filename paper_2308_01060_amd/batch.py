"""Many independent scenes stepped together: one launch per phase for all of them.

``BatchedParticleSet`` holds the flattened particle arrays of every scene
(scene k owns particles [p_offset_k, p_offset_k + n_k)) and their grids laid
end to end, and runs the batched entry points of the library:

    polypic_batch_sort -> polypic_batch_p2g -> polypic_batch_grid_update
                       -> polypic_batch_g2p (+ advection)

From the second step on the sort is the exact re-sort from the previous step's
keys (``polypic_batch_sort_update``), as in ``ParticleSet``.  Fused (the default),
the G2P of a step and the P2G of the next are one call,
``polypic_batch_g2p2g``, as in ``ParticleSet``: a step is sort -> grid update ->
G2P2G, with a P2G first when the grid does not hold the current state.

Fused steps keep the grid passes to the active regions (16 x 4 x 4-node boxes)
that the previous G2P2G flagged: after the first step, the grid update is
``polypic_batch_grid_update_active`` (which also clears the grid) and G2P2G adds
into the cleared grid, flagging where it lands.

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
                 device: str = "cuda", fused: bool = True, incremental_sort: bool = True):
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
        # incremental re-sort, as in ParticleSet: slot_keys[i] = the key slot i was sorted under
        self.incremental_sort = bool(incremental_sort)
        self.slot_keys = torch.empty_like(self.keys) if self.incremental_sort else None
        self.slot_keys_valid = False
        self._keys_are_slot_keys = False
        self.resort_ws = (torch.empty(max(1, ops.polypic_batch_sort_update_workspace_bytes(
            self.batch)), dtype=torch.uint8, device=device) if self.incremental_sort else None)
        self.status = torch.zeros(1, dtype=torch.int32, device=device)
        self.graphs = None
        self.phase = 0
        self.fused = bool(fused)
        self.grid_current = False  # grid_mass / grid_mom hold the P2G of the current state
        self._next_grid_current = False
        # active regions: the fused scatter flags them; regions_valid says that grid_mass /
        # grid_mom are zero outside the flagged regions (the last writer was a flagging G2P2G)
        self.region_state = torch.zeros(ops.region_state_words(self.batch.n_regions),
                                        dtype=torch.int32, device=device)
        self.regions_valid = False

    @property
    def P(self) -> int:
        return self.batch.P

    def scene_slice(self, k: int) -> slice:
        return slice(self.batch.p_offsets[k], self.batch.p_offsets[k + 1])

    def node_slice(self, k: int) -> slice:
        return slice(self.batch.node_offsets[k], self.batch.node_offsets[k + 1])

    # ---- phases
    def _take_slot_keys(self):
        """After a step in sort order, `keys` describes the slot order: make it slot_keys."""
        if self._keys_are_slot_keys:
            self.keys, self.slot_keys = self.slot_keys, self.keys
            self._keys_are_slot_keys = False
            self.slot_keys_valid = True

    def sort(self, full: bool = False):
        """Every scene's cell-key sort: the exact re-sort from the keys the slot order was
        sorted under when they are known, else (or with full=True) the full sort."""
        self._take_slot_keys()
        if self.slot_keys_valid and not full:
            ops.polypic_batch_sort_update(self.batch, self.x, self.slot_keys, self.keys,
                                          self.perm, self.resort_ws, self.status)
        else:
            ops.polypic_batch_sort(self.batch, self.x, self.keys, self.perm, self.sort_ws,
                                   self.status)

    def p2g(self, use_perm: bool = True):
        ops.polypic_batch_p2g(self.batch, self.n_modes, self.x, self.coeff, self.grid_mass,
                              self.grid_mom, mass=self.mass, uniform_mass=self.uniform_mass,
                              perm=self.perm if use_perm else None, status_dev=self.status)
        self.grid_current = True
        self.regions_valid = False

    def grid_update(self):
        ops.polypic_batch_grid_update(self.batch, self.dt, self.gravity, self.bc_layers,
                                      self.grid_mass, self.grid_mom, self.grid_vel)

    def grid_update_active(self):
        """The grid update on the flagged regions only; it leaves the grid cleared."""
        if not self.regions_valid:
            raise RuntimeError("the grid is not confined to flagged regions")
        ops.polypic_batch_grid_update_active(self.batch, self.dt, self.gravity, self.bc_layers,
                                             self.grid_mass, self.grid_mom, self.grid_vel,
                                             self.region_state)

    def g2p(self, use_perm: bool = True):
        ops.polypic_batch_g2p(self.batch, self.n_modes, self.dt, self.grid_vel, self.x,
                              self.coeff_next, perm=self.perm if use_perm else None,
                              x_out=self.x_next, mass_in=self.mass, mass_out=self.mass_next,
                              status_dev=self.status)
        self._next_grid_current = False

    def g2p2g(self, use_perm: bool = True, accumulate: bool = False):
        """G2P + advection of every scene, and the P2G of the new state into the grid
        (cleared first, or with accumulate=True added to a grid the active update cleared),
        flagging the regions it lands in."""
        ops.polypic_batch_g2p2g(self.batch, self.n_modes, self.dt, self.grid_vel, self.x,
                                self.x_next, self.coeff_next, self.grid_mass, self.grid_mom,
                                perm=self.perm if use_perm else None, mass_in=self.mass,
                                mass_out=self.mass_next, uniform_mass=self.uniform_mass,
                                status_dev=self.status, accumulate=accumulate,
                                region_state=self.region_state)
        self._next_grid_current = True
        self.regions_valid = True

    def swap(self):
        self.x, self.x_next = self.x_next, self.x
        if self.mass is not None:
            self.mass, self.mass_next = self.mass_next, self.mass
        self.grid_current = self._next_grid_current
        self._next_grid_current = False
        # G2P wrote slot i from particle perm[i]: slot i was sorted under keys[i]
        if self.incremental_sort:
            self._keys_are_slot_keys = True

    def _step_calls(self):
        """One step after the sort, the grid holding the current state's P2G when fused."""
        if self.fused:
            if self.regions_valid:
                self.grid_update_active()
                self.g2p2g(accumulate=True)
            else:
                self.grid_update()
                self.g2p2g()
        else:
            self.p2g()
            self.grid_update()
            self.g2p()

    def step(self):
        """One eager step for every scene (outputs come out in each scene's cell order)."""
        self.sort()
        if self.fused and not self.grid_current:
            self.p2g()  # the first step's P2G; later ones come from the G2P2G before them
        self._step_calls()
        self.swap()
        self.phase ^= 1

    def invalidate_grid(self):
        """Call after changing x, coeff or mass directly: the next fused step redoes P2G."""
        self.grid_current = False

    def autotune(self):
        """Sort, then let the library time its batched P2G configurations (synchronises)."""
        self.sort()
        self.regions_valid = False  # the timed P2G calls rewrite the grid
        return ops.polypic_batch_autotune(self.batch, self.n_modes, self.x, self.coeff,
                                          self.grid_mass, self.grid_mom, mass=self.mass,
                                          uniform_mass=self.uniform_mass, perm=self.perm)

    # ---- graph capture
    def capture(self):
        """Capture one step in each buffer direction as a HIP graph.

        Fused, the graphs hold sort -> active grid update -> G2P2G, so the grid must hold
        the current state's P2G, confined to flagged regions, before the first replay: one
        eager step does that, and capture runs one itself when the grid holds the current
        state but its regions are not known (after the autotuner's P2G calls)."""
        if self.fused and not self.grid_current:
            raise RuntimeError("fused capture needs the grid current: run one step() first")
        if self.fused and not self.regions_valid:
            self.step()
        torch.cuda.synchronize()
        graphs = []
        for _ in range(2):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                self.sort()
                self._step_calls()
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
        # the bookkeeping of what the graph ran: its sort (key roles) and its last call
        self._take_slot_keys()
        self._next_grid_current = self.fused  # the graph ends with G2P2G (fused) or G2P
        self.swap()
        self.phase ^= 1

    def status_flags(self) -> int:
        return int(self.status.item())
