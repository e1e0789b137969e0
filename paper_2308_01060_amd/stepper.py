"""A particle set on its grid, stepped through the C ABI.

``ParticleSet`` owns the device buffers of one particle set (double-buffered
positions / coefficients / optional mass and F), its grid arrays and the sort
workspace, and runs one transfer step as four library calls on the current
stream:

    polypic_sort -> polypic_p2g -> polypic_grid_update -> polypic_g2p

or, fused (the default), ``polypic_g2p2g`` in place of the G2P of one step and the
P2G of the next: G2P reads no coefficients, and the next P2G is their only reader,
so the new state is scattered into the grid while its coefficients are still in
registers (a step is then sort -> grid update -> G2P2G).

G2P writes the new state in sorted order, so after a step the arrays are in
cell order and the next sort is close to the identity: from the second step on,
``sort`` re-sorts incrementally (``polypic_sort_update``: only the particles
whose cell changed are sorted, then merged; same result as a full sort).  G2P reads no
coefficients, so by default it writes the new ones over the array P2G read
(``coeff_in_place``): one coefficient array instead of two (1.4 GB saved at
27 modes and 4.19 M particles).  The set takes ownership of the tensors it is
given and overwrites them as it steps.  ``order`` (int32) tracks the
original index of each slot (one polypic_gather_rows per step; switch it off
with ``track_order=False`` when only the transfers matter).
"""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from . import ops


class ParticleSet:
    def __init__(self, grid, n_modes: int, x: torch.Tensor, coeff: torch.Tensor,
                 mass: Optional[torch.Tensor] = None, uniform_mass: float = 1.0,
                 F: Optional[torch.Tensor] = None, dt: float = 1e-4,
                 gravity: Sequence[float] = (0.0, -9.8, 0.0), bc_layers: int = 1,
                 device: str = "cuda", track_order: bool = True, coeff_in_place: bool = True,
                 incremental_sort: bool = True, fused: bool = True):
        if n_modes not in ops.ALLOWED_N_MODES:
            raise ValueError("n_modes must be one of 1, 4, 8, 27")
        self.grid = grid
        self.n_modes = int(n_modes)
        self.dt = float(dt)
        self.gravity = tuple(float(g) for g in gravity)
        self.bc_layers = int(bc_layers)
        self.uniform_mass = float(uniform_mass)
        P = int(x.shape[-1])
        self.P = P
        dev = torch.device(device)
        f32 = dict(dtype=torch.float32, device=dev)
        self.x = x.to(**f32).contiguous().reshape(3, P)
        c = coeff.to(**f32)
        if c.shape[1] != self.n_modes:
            c = c[:, : self.n_modes]
        self.coeff = c.contiguous()
        self.mass = None if mass is None else mass.to(**f32).contiguous()
        self.F = None if F is None else F.to(**f32).contiguous().reshape(9, P)
        self.x_next = torch.empty_like(self.x)
        self.coeff_in_place = bool(coeff_in_place)
        self.coeff_next = self.coeff if self.coeff_in_place else torch.empty_like(self.coeff)
        self.mass_next = None if self.mass is None else torch.empty_like(self.mass)
        self.F_next = None if self.F is None else torch.empty_like(self.F)
        N = ops.n_nodes(grid)
        self.grid_mass = torch.empty(N, **f32)
        self.grid_mom = torch.empty(3 * N, **f32)
        self.grid_vel = torch.empty(3 * N, **f32)
        self.keys = torch.empty(P, dtype=torch.int32, device=dev)
        self.perm = torch.empty(P, dtype=torch.int32, device=dev)
        self.ws = torch.empty(max(1, ops.polypic_sort_workspace_bytes(grid, P)),
                              dtype=torch.uint8, device=dev)
        # incremental re-sort: slot_keys[i] = the key slot i of the particle arrays was sorted
        # under (valid once a step has permuted the arrays by a sort), and its workspace
        self.incremental_sort = bool(incremental_sort)
        self.slot_keys = torch.empty_like(self.keys) if self.incremental_sort else None
        self.slot_keys_valid = False
        self._keys_are_slot_keys = False  # set by swap(): `keys` now describes the slot order
        self.resort_ws = (torch.empty(max(1, ops.polypic_sort_update_workspace_bytes(grid, P)),
                                      dtype=torch.uint8, device=dev)
                          if self.incremental_sort else None)
        self.p2g_ws = torch.empty(max(1, ops.polypic_p2g_workspace_bytes(grid, P)),
                                  dtype=torch.uint8, device=dev)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        self.track_order = bool(track_order)
        self.order = torch.arange(P, dtype=torch.int32, device=dev)
        # fused stepping: G2P scatters the new state into the grid at once (polypic_g2p2g);
        # grid_current says grid_mass / grid_mom hold the P2G of the current state
        self.fused = bool(fused)
        self.grid_current = False
        self._next_grid_current = False
        # active regions (16 x 4 x 4-node boxes): the fused scatter flags where it lands;
        # regions_valid says that grid_mass / grid_mom are zero outside the flagged regions
        # (their last writer was a flagging G2P2G), so the grid update may visit those only
        self.region_state = torch.zeros(
            ops.region_state_words(ops.polypic_region_count(grid)), dtype=torch.int32,
            device=dev)
        self.regions_valid = False

    # -- the four calls of one step
    def sort(self, full: bool = False):
        """Cell-key sort of the current positions into keys / perm: the exact re-sort from
        the keys the current slot order was sorted under when they are known, else (or with
        full=True) the full sort.  Both give the same result."""
        if self._keys_are_slot_keys:
            self.keys, self.slot_keys = self.slot_keys, self.keys
            self._keys_are_slot_keys = False
            self.slot_keys_valid = True
        if self.slot_keys_valid and not full:
            ops.polypic_sort_update(self.grid, self.x, self.slot_keys, self.keys, self.perm,
                                    self.resort_ws, self.status)
        else:
            ops.polypic_sort(self.grid, self.x, self.keys, self.perm, self.ws, self.status)

    def p2g(self, use_perm: bool = True, use_keys: bool = True):
        """P2G in sort order (use_perm); use_keys hands the sorted keys over as well, which the
        cell-run path needs when the configuration table selects it."""
        sorted_ = use_perm and use_keys
        ops.polypic_p2g(self.grid, self.n_modes, self.x, self.coeff, self.grid_mass,
                        self.grid_mom, mass=self.mass, uniform_mass=self.uniform_mass,
                        perm=self.perm if use_perm else None,
                        keys_sorted=self.keys if sorted_ else None,
                        ws=self.p2g_ws if sorted_ else None, status_dev=self.status)
        self.grid_current = True
        self.regions_valid = False

    def autotune(self):
        """Sort, then let the library time its P2G configurations on this set (synchronises)."""
        self.sort()
        self.regions_valid = False
        return ops.polypic_autotune_p2g(self.grid, self.n_modes, self.x, self.coeff, self.grid_mass,
                                        self.grid_mom, mass=self.mass,
                                        uniform_mass=self.uniform_mass, perm=self.perm,
                                        keys_sorted=self.keys, ws=self.p2g_ws)

    def grid_update(self, clear: bool = False):
        """Grid velocities from grid_mass / grid_mom; with clear=True those two are zeroed
        once read (polypic_grid_update_clear), ready for g2p2g(accumulate=True)."""
        fn = ops.polypic_grid_update_clear if clear else ops.polypic_grid_update
        fn(self.grid, self.dt, self.gravity, self.bc_layers, self.grid_mass, self.grid_mom,
           self.grid_vel)
        if clear:
            self.grid_current = False

    def grid_update_active(self):
        """The grid update with clearing, on the regions the last G2P2G flagged only."""
        if not self.regions_valid:
            raise RuntimeError("the grid is not confined to flagged regions")
        ops.polypic_grid_update_active(self.grid, self.dt, self.gravity, self.bc_layers,
                                       self.grid_mass, self.grid_mom, self.grid_vel,
                                       self.region_state)
        self.grid_current = False

    def autotune_fused(self):
        """One step in which the library times the fused G2P2G's lane groups and chunk orders
        on this set and keeps the fastest for later calls at this mode count (synchronises);
        returns it (ops.FusedChoice)."""
        self.sort()
        if not self.grid_current:
            self.p2g()
        self.grid_update()
        choice = ops.polypic_autotune_g2p2g(self.grid, self.n_modes, self.dt, self.grid_vel,
                                            self.x, self.x_next, self.coeff_next, self.grid_mass,
                                            self.grid_mom, perm=self.perm, F_in=self.F,
                                            F_out=self.F_next, mass_in=self.mass,
                                            mass_out=self.mass_next,
                                            uniform_mass=self.uniform_mass)
        self._next_grid_current = True
        self.regions_valid = False  # the timed calls flag nothing
        self.swap()
        return choice

    def g2p(self, use_perm: bool = True, advect: bool = True):
        ops.polypic_g2p(self.grid, self.n_modes, self.dt, self.grid_vel, self.x, self.coeff_next,
                        perm=self.perm if use_perm else None,
                        x_out=self.x_next if advect else None,
                        F_in=self.F, F_out=self.F_next,
                        mass_in=self.mass, mass_out=self.mass_next, status_dev=self.status)
        self._next_grid_current = False

    def g2p2g(self, use_perm: bool = True, accumulate: bool = False):
        """G2P + advection, and the P2G of the new state into grid_mass / grid_mom (the grid
        velocity has been computed from them already).  accumulate=True adds to the two
        (zeroed by a clearing grid update) instead of clearing them first.  The regions the
        scatter lands in are flagged."""
        ops.polypic_g2p2g(self.grid, self.n_modes, self.dt, self.grid_vel, self.x, self.x_next,
                          self.coeff_next, self.grid_mass, self.grid_mom,
                          perm=self.perm if use_perm else None, F_in=self.F, F_out=self.F_next,
                          mass_in=self.mass, mass_out=self.mass_next,
                          uniform_mass=self.uniform_mass, status_dev=self.status,
                          accumulate=accumulate, region_state=self.region_state)
        self._next_grid_current = True
        self.regions_valid = True

    def invalidate_grid(self):
        """Call after changing x, coeff or mass directly: the next fused step redoes P2G."""
        self.grid_current = False

    def swap(self, use_perm: bool = True):
        self.x, self.x_next = self.x_next, self.x
        if not self.coeff_in_place:
            self.coeff, self.coeff_next = self.coeff_next, self.coeff
        if self.mass is not None:
            self.mass, self.mass_next = self.mass_next, self.mass
        if self.F is not None:
            self.F, self.F_next = self.F_next, self.F
        if use_perm and self.track_order:
            order = torch.empty_like(self.order)
            ops.polypic_gather_rows(self.order, order, self.perm)
            self.order = order
        # G2P wrote slot i from particle perm[i]: slot i was sorted under keys[i].  (Without
        # the permutation the slot order is unchanged, and so is what describes it.)
        if self.incremental_sort and use_perm:
            self._keys_are_slot_keys = True
        self.grid_current = self._next_grid_current
        self._next_grid_current = False

    def step(self):
        """One full step: sort, P2G, grid update, G2P + advection, then swap buffers.  Fused
        (default), the P2G of a step was done by the G2P of the step before (polypic_g2p2g),
        so a step is sort, grid update, G2P2G -- with a P2G first when the grid is not
        current (the first step).  The grid update zeroes the sums it read, and G2P2G adds
        into them, so the grid is not cleared in a pass of its own; once a G2P2G has flagged
        the regions it scattered into, the update visits those regions only."""
        self.sort()
        if self.fused:
            if not self.grid_current:
                self.p2g()
            if self.regions_valid:
                self.grid_update_active()
            else:
                self.grid_update(clear=True)
            self.g2p2g(accumulate=True)
        else:
            self.p2g()
            self.grid_update()
            self.g2p()
        self.swap()

    def status_flags(self) -> int:
        return int(self.status.item())


class MacParticleSet(ParticleSet):
    """A particle set on a staggered (MAC) grid: component a of the velocity on its own
    faces, each face with its own mass (three face-mass arrays instead of one node mass).

    A step is sort -> polypic_mac_p2g -> polypic_mac_grid_update -> polypic_mac_g2p
    (separate calls; the sort and re-sort, buffer swaps and order tracking are those of
    ParticleSet: the cell key of the node stencil also orders the face stencils)."""

    def __init__(self, grid, n_modes: int, x: torch.Tensor, coeff: torch.Tensor, **kw):
        kw["fused"] = False
        super().__init__(grid, n_modes, x, coeff, **kw)
        N = ops.n_nodes(grid)
        dev = self.x.device
        self.grid_mass = torch.empty(3 * N, dtype=torch.float32, device=dev)  # face masses

    def p2g(self, use_perm: bool = True, use_keys: bool = True):
        ops.polypic_mac_p2g(self.grid, self.n_modes, self.x, self.coeff, self.grid_mass,
                            self.grid_mom, mass=self.mass, uniform_mass=self.uniform_mass,
                            perm=self.perm if use_perm else None, status_dev=self.status)
        self.grid_current = True

    def autotune(self):
        """The MAC kernels have one configuration: only the sort runs."""
        self.sort()
        return None

    def grid_update(self, clear: bool = False):
        if clear:
            raise RuntimeError("no clearing grid update for this set (it steps unfused)")
        ops.polypic_mac_grid_update(self.grid, self.dt, self.gravity, self.bc_layers,
                                    self.grid_mass, self.grid_mom, self.grid_vel)

    def g2p(self, use_perm: bool = True, advect: bool = True):
        ops.polypic_mac_g2p(self.grid, self.n_modes, self.dt, self.grid_vel, self.x,
                            self.coeff_next, perm=self.perm if use_perm else None,
                            x_out=self.x_next if advect else None, F_in=self.F, F_out=self.F_next,
                            mass_in=self.mass, mass_out=self.mass_next, status_dev=self.status)
        self._next_grid_current = False

    def g2p2g(self, use_perm: bool = True):
        raise RuntimeError("a MAC set steps with separate P2G and G2P calls (fused=False)")


class AffineParticleSet(ParticleSet):
    """A particle set whose P2G evaluates the modes through the affine back-map of Eq. 12
    (polypic_p2g_affine): the coefficients a G2P fitted at the positions x^n are carried
    to the grid from x^{n+1} at z' = (I + dt C)^-1 (x_i - x^{n+1}) / dx, with the quadratic
    factor of x^n.  The set keeps x^n in slot order beside the positions (x_fit: one
    polypic_gather_rows of 3 rows per step).  The first step's coefficients count as
    fitted at the initial positions (plain P2G).  Separate P2G and G2P calls."""

    def __init__(self, grid, n_modes: int, x: torch.Tensor, coeff: torch.Tensor, **kw):
        kw["fused"] = False
        super().__init__(grid, n_modes, x, coeff, **kw)
        self.x_fit = torch.empty_like(self.x)
        self.x_fit_next = torch.empty_like(self.x)
        self.fit_valid = False
        self._next_fit_valid = False

    def p2g(self, use_perm: bool = True, use_keys: bool = True):
        if not self.fit_valid:
            return super().p2g(use_perm, use_keys)
        ops.polypic_p2g_affine(self.grid, self.n_modes, self.dt, self.x, self.coeff,
                               self.grid_mass, self.grid_mom, x_fit=self.x_fit, mass=self.mass,
                               uniform_mass=self.uniform_mass,
                               perm=self.perm if use_perm else None, status_dev=self.status)
        self.grid_current = True

    def g2p(self, use_perm: bool = True, advect: bool = True):
        super().g2p(use_perm, advect)
        # the new coefficients are fitted at the present positions, slot i at x[perm[i]]
        if use_perm:
            ops.polypic_gather_rows(self.x, self.x_fit_next, self.perm)
        else:
            self.x_fit_next.copy_(self.x)
        self._next_fit_valid = True

    def g2p2g(self, use_perm: bool = True):
        raise RuntimeError("an affine-map set steps with separate P2G and G2P calls")

    def swap(self, use_perm: bool = True):
        super().swap(use_perm)
        self.x_fit, self.x_fit_next = self.x_fit_next, self.x_fit
        self.fit_valid = self._next_fit_valid
        self._next_fit_valid = False


class MixtureParticleSet(ParticleSet):
    """Liquid and fabric particles in one array on one grid (section 3.4): per particle a
    phase (0 fluid, 1 solid), the fluid mass m_f (for a solid point, its absorbed fluid)
    and the solid mass m_s; the grid holds a fluid and a solid set of channels
    (grid_mass [2][N], grid_mom and grid_vel [2][3][N]).  A step is sort ->
    polypic_mixture_p2g -> polypic_mixture_grid_update -> polypic_mixture_g2p, and the
    per-particle arrays follow the sort like the positions."""

    def __init__(self, grid, n_modes: int, x: torch.Tensor, coeff: torch.Tensor,
                 phase: torch.Tensor, mass_f: torch.Tensor,
                 mass_s: Optional[torch.Tensor] = None, **kw):
        kw["fused"] = False
        kw.pop("mass", None)
        super().__init__(grid, n_modes, x, coeff, **kw)
        dev = self.x.device
        N = ops.n_nodes(grid)
        f32 = dict(dtype=torch.float32, device=dev)
        self.phase = phase.to(dtype=torch.int32, device=dev).contiguous()
        self.mass_f = mass_f.to(**f32).contiguous()
        self.mass_s = None if mass_s is None else mass_s.to(**f32).contiguous()
        self.phase_next = torch.empty_like(self.phase)
        self.mass_f_next = torch.empty_like(self.mass_f)
        self.mass_s_next = None if self.mass_s is None else torch.empty_like(self.mass_s)
        self.grid_mass = torch.empty(2 * N, **f32)
        self.grid_mom = torch.empty(6 * N, **f32)
        self.grid_vel = torch.empty(6 * N, **f32)

    def p2g(self, use_perm: bool = True, use_keys: bool = True):
        ops.polypic_mixture_p2g(self.grid, self.n_modes, self.x, self.phase, self.mass_f,
                                self.coeff, self.grid_mass, self.grid_mom, mass_s=self.mass_s,
                                perm=self.perm if use_perm else None, status_dev=self.status)
        self.grid_current = True

    def autotune(self):
        """The mixture kernels have one configuration: only the sort runs."""
        self.sort()
        return None

    def grid_update(self, clear: bool = False):
        if clear:
            raise RuntimeError("no clearing grid update for this set (it steps unfused)")
        ops.polypic_mixture_grid_update(self.grid, self.dt, self.gravity, self.bc_layers,
                                        self.grid_mass, self.grid_mom, self.grid_vel)

    def g2p(self, use_perm: bool = True, advect: bool = True):
        ops.polypic_mixture_g2p(self.grid, self.n_modes, self.dt, self.grid_vel, self.x,
                                self.phase, self.coeff_next,
                                perm=self.perm if use_perm else None,
                                x_out=self.x_next if advect else None, F_in=self.F,
                                F_out=self.F_next, phase_out=self.phase_next,
                                mass_f_in=self.mass_f, mass_f_out=self.mass_f_next,
                                mass_s_in=self.mass_s, mass_s_out=self.mass_s_next,
                                status_dev=self.status)
        self._next_grid_current = False

    def g2p2g(self, use_perm: bool = True):
        raise RuntimeError("a mixture set steps with separate P2G and G2P calls")

    def swap(self, use_perm: bool = True):
        super().swap(use_perm)
        self.phase, self.phase_next = self.phase_next, self.phase
        self.mass_f, self.mass_f_next = self.mass_f_next, self.mass_f
        if self.mass_s is not None:
            self.mass_s, self.mass_s_next = self.mass_s_next, self.mass_s
