"""Torch-facing binding of the C ABI: same entry-point names, argument marshalling only.

Tensors must be CUDA (HIP) float32 / int32 / uint32 tensors, contiguous, with
the layouts of include/polypic.h.  Work is enqueued on torch's current stream;
nothing here computes any part of the transfers.
"""
from __future__ import annotations

import ctypes
from typing import List, NamedTuple, Optional, Sequence, Tuple

import torch

from . import _lib
from ._lib import check, polypic_grid

ALLOWED_N_MODES = (1, 4, 8, 27)


def make_grid(nodes: Sequence[int], dx: float, origin: Sequence[float] = (0.0, 0.0, 0.0),
              inv_dx: Optional[float] = None) -> polypic_grid:
    """Build the C grid struct; inv_dx defaults to 1/dx rounded to float32."""
    g = polypic_grid()
    g.nx, g.ny, g.nz = (int(n) for n in nodes)
    g.dx = float(dx)
    g.inv_dx = float(1.0 / dx if inv_dx is None else inv_dx)
    for a in range(3):
        g.origin[a] = float(origin[a])
    return g


def grid_from_spec(spec) -> polypic_grid:
    """C grid struct from a workloads.GridSpec (duck-typed: nodes, dx, inv_dx, origin)."""
    return make_grid(spec.nodes, spec.dx, spec.origin, spec.inv_dx)


def n_nodes(g: polypic_grid) -> int:
    return int(g.nx) * int(g.ny) * int(g.nz)


def _stream() -> int:
    return int(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor], dtype: torch.dtype, numel: int, name: str) -> Optional[int]:
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return t.data_ptr()


def polypic_sort_workspace_bytes(grid: polypic_grid, P: int) -> int:
    out = ctypes.c_size_t(0)
    check(_lib.load().polypic_sort_workspace_bytes(ctypes.byref(grid), int(P), ctypes.byref(out)),
          "polypic_sort_workspace_bytes")
    return int(out.value)


def _keys_ptr(keys: Optional[torch.Tensor], P: int) -> Optional[int]:
    """Cell keys are uint32 in the C ABI; an int32 tensor holds the same bits."""
    if keys is None:
        return None
    dtype = torch.int32 if keys.dtype == torch.int32 else torch.uint32
    return _ptr(keys, dtype, P, "keys")


def polypic_sort(grid: polypic_grid, x: torch.Tensor, keys_out: torch.Tensor,
                 perm_out: torch.Tensor, ws: torch.Tensor,
                 status_dev: Optional[torch.Tensor] = None) -> None:
    P = x.numel() // 3
    check(_lib.load().polypic_sort(
        ctypes.byref(grid), P, _ptr(x, torch.float32, 3 * P, "x"),
        _keys_ptr(keys_out, P),
        _ptr(perm_out, torch.int32, P, "perm_out"),
        _ptr(ws, torch.uint8, ws.numel(), "ws"), ws.numel(),
        _ptr(status_dev, torch.int32, 1, "status_dev"), _stream()), "polypic_sort")


def polypic_sort_noalloc(grid: polypic_grid, x: torch.Tensor, keys_out: torch.Tensor,
                         perm_out: torch.Tensor,
                         status_dev: Optional[torch.Tensor] = None) -> None:
    """polypic_sort with the library's static device workspace (no ws argument, nothing
    allocated); at most POLYPIC_SORT_NOALLOC_MAX_P particles."""
    P = x.numel() // 3
    check(_lib.load().polypic_sort_noalloc(
        ctypes.byref(grid), P, _ptr(x, torch.float32, 3 * P, "x"),
        _keys_ptr(keys_out, P),
        _ptr(perm_out, torch.int32, P, "perm_out"),
        _ptr(status_dev, torch.int32, 1, "status_dev"), _stream()), "polypic_sort_noalloc")


def polypic_sort_update_workspace_bytes(grid: polypic_grid, P: int) -> int:
    out = ctypes.c_size_t(0)
    check(_lib.load().polypic_sort_update_workspace_bytes(ctypes.byref(grid), int(P),
                                                          ctypes.byref(out)),
          "polypic_sort_update_workspace_bytes")
    return int(out.value)


def polypic_sort_update(grid: polypic_grid, x: torch.Tensor, keys_prev: torch.Tensor,
                        keys_out: torch.Tensor, perm_out: torch.Tensor, ws: torch.Tensor,
                        status_dev: Optional[torch.Tensor] = None) -> None:
    """Re-sort after a step (keys_prev: the previous sort's keys, in the current slot order)."""
    P = x.numel() // 3
    check(_lib.load().polypic_sort_update(
        ctypes.byref(grid), P, _ptr(x, torch.float32, 3 * P, "x"), _keys_ptr(keys_prev, P),
        _keys_ptr(keys_out, P), _ptr(perm_out, torch.int32, P, "perm_out"),
        _ptr(ws, torch.uint8, ws.numel(), "ws"), ws.numel(),
        _ptr(status_dev, torch.int32, 1, "status_dev"), _stream()), "polypic_sort_update")


def polypic_p2g_workspace_bytes(grid: polypic_grid, P: int) -> int:
    out = ctypes.c_size_t(0)
    check(_lib.load().polypic_p2g_workspace_bytes(ctypes.byref(grid), int(P), ctypes.byref(out)),
          "polypic_p2g_workspace_bytes")
    return int(out.value)


def polypic_p2g(grid: polypic_grid, n_modes: int, x: torch.Tensor, coeff: torch.Tensor,
                grid_mass: torch.Tensor, grid_mom: torch.Tensor,
                mass: Optional[torch.Tensor] = None, uniform_mass: float = 1.0,
                perm: Optional[torch.Tensor] = None, keys_sorted: Optional[torch.Tensor] = None,
                ws: Optional[torch.Tensor] = None, accumulate: bool = False,
                status_dev: Optional[torch.Tensor] = None) -> None:
    P = x.numel() // 3
    N = n_nodes(grid)
    check(_lib.load().polypic_p2g(
        ctypes.byref(grid), P, int(n_modes), _ptr(x, torch.float32, 3 * P, "x"),
        _ptr(mass, torch.float32, P, "mass"), float(uniform_mass),
        _ptr(coeff, torch.float32, 3 * int(n_modes) * P, "coeff"),
        _ptr(perm, torch.int32, P, "perm"), _keys_ptr(keys_sorted, P),
        _ptr(ws, torch.uint8, ws.numel() if ws is not None else 0, "ws"),
        0 if ws is None else ws.numel(),
        _ptr(grid_mass, torch.float32, N, "grid_mass"),
        _ptr(grid_mom, torch.float32, 3 * N, "grid_mom"), int(bool(accumulate)),
        _ptr(status_dev, torch.int32, 1, "status_dev"), _stream()), "polypic_p2g")


class P2GChoice(NamedTuple):
    """A P2G launch configuration (include/polypic.h): path, workgroup size, chunk schedule,
    persistent workgroups per CU, brick edge in cells."""

    path: int
    block: int
    schedule: int = _lib.POLYPIC_SCHED_LINEAR
    per_cu: int = 0
    brick: int = 4


def polypic_set_p2g_config(n_modes: int, path: int, block: int = 512,
                           schedule: int = _lib.POLYPIC_SCHED_LINEAR, per_cu: int = 0,
                           brick: int = 4) -> None:
    check(_lib.load().polypic_set_p2g_config(int(n_modes), int(path), int(block), int(schedule),
                                             int(per_cu), int(brick)), "polypic_set_p2g_config")


def polypic_get_p2g_config(n_modes: int) -> P2GChoice:
    v = [ctypes.c_int32(0) for _ in range(5)]
    check(_lib.load().polypic_get_p2g_config(int(n_modes), *[ctypes.byref(t) for t in v]),
          "polypic_get_p2g_config")
    return P2GChoice(*(int(t.value) for t in v))


def polypic_autotune_p2g(grid: polypic_grid, n_modes: int, x: torch.Tensor, coeff: torch.Tensor,
                         grid_mass: torch.Tensor, grid_mom: torch.Tensor,
                         mass: Optional[torch.Tensor] = None, uniform_mass: float = 1.0,
                         perm: Optional[torch.Tensor] = None,
                         keys_sorted: Optional[torch.Tensor] = None,
                         ws: Optional[torch.Tensor] = None) -> P2GChoice:
    """Times every P2G configuration on these inputs; returns the chosen one."""
    P = x.numel() // 3
    N = n_nodes(grid)
    v = [ctypes.c_int32(0) for _ in range(5)]
    check(_lib.load().polypic_autotune_p2g(
        ctypes.byref(grid), P, int(n_modes), _ptr(x, torch.float32, 3 * P, "x"),
        _ptr(mass, torch.float32, P, "mass"), float(uniform_mass),
        _ptr(coeff, torch.float32, 3 * int(n_modes) * P, "coeff"),
        _ptr(perm, torch.int32, P, "perm"), _keys_ptr(keys_sorted, P),
        _ptr(ws, torch.uint8, ws.numel() if ws is not None else 0, "ws"),
        0 if ws is None else ws.numel(),
        _ptr(grid_mass, torch.float32, N, "grid_mass"),
        _ptr(grid_mom, torch.float32, 3 * N, "grid_mom"),
        *[ctypes.byref(t) for t in v], _stream()), "polypic_autotune_p2g")
    return P2GChoice(*(int(t.value) for t in v))


def polypic_set_g2p_schedule(schedule: int) -> None:
    check(_lib.load().polypic_set_g2p_schedule(int(schedule)), "polypic_set_g2p_schedule")


def polypic_get_g2p_schedule() -> int:
    v = ctypes.c_int32(0)
    check(_lib.load().polypic_get_g2p_schedule(ctypes.byref(v)), "polypic_get_g2p_schedule")
    return int(v.value)


def polypic_grid_update(grid: polypic_grid, dt: float, gravity: Sequence[float], bc_layers: int,
                        grid_mass: torch.Tensor, grid_mom: torch.Tensor,
                        grid_vel: torch.Tensor) -> None:
    N = n_nodes(grid)
    g3 = (ctypes.c_float * 3)(*[float(v) for v in gravity])
    check(_lib.load().polypic_grid_update(
        ctypes.byref(grid), float(dt), g3, int(bc_layers),
        _ptr(grid_mass, torch.float32, N, "grid_mass"),
        _ptr(grid_mom, torch.float32, 3 * N, "grid_mom"),
        _ptr(grid_vel, torch.float32, 3 * N, "grid_vel"), _stream()), "polypic_grid_update")


def polypic_grid_update_clear(grid: polypic_grid, dt: float, gravity: Sequence[float],
                              bc_layers: int, grid_mass: torch.Tensor, grid_mom: torch.Tensor,
                              grid_vel: torch.Tensor) -> None:
    """polypic_grid_update that zeroes grid_mass and grid_mom once read."""
    N = n_nodes(grid)
    g3 = (ctypes.c_float * 3)(*[float(v) for v in gravity])
    check(_lib.load().polypic_grid_update_clear(
        ctypes.byref(grid), float(dt), g3, int(bc_layers),
        _ptr(grid_mass, torch.float32, N, "grid_mass"),
        _ptr(grid_mom, torch.float32, 3 * N, "grid_mom"),
        _ptr(grid_vel, torch.float32, 3 * N, "grid_vel"), _stream()),
        "polypic_grid_update_clear")


def region_state_words(n_regions: int) -> int:
    """uint32 words of a region state: one flag per region."""
    return int(n_regions)


def _regions_ptr(state: Optional[torch.Tensor], n_regions: int) -> Optional[int]:
    """The region state is uint32 in the C ABI; an int32 tensor holds the same bits."""
    return _ptr(state, torch.int32, region_state_words(n_regions), "region_state")


def polypic_region_count(grid: polypic_grid) -> int:
    """Active regions of a grid (boxes of 16 x 4 x 4 nodes)."""
    out = ctypes.c_int64(0)
    check(_lib.load().polypic_region_count(ctypes.byref(grid), ctypes.byref(out)),
          "polypic_region_count")
    return int(out.value)


def polypic_grid_update_active(grid: polypic_grid, dt: float, gravity: Sequence[float],
                               bc_layers: int, grid_mass: torch.Tensor, grid_mom: torch.Tensor,
                               grid_vel: torch.Tensor, region_state: torch.Tensor) -> None:
    """polypic_grid_update_clear on the flagged regions only; resets their flags."""
    N = n_nodes(grid)
    g3 = (ctypes.c_float * 3)(*[float(v) for v in gravity])
    check(_lib.load().polypic_grid_update_active(
        ctypes.byref(grid), float(dt), g3, int(bc_layers),
        _ptr(grid_mass, torch.float32, N, "grid_mass"),
        _ptr(grid_mom, torch.float32, 3 * N, "grid_mom"),
        _ptr(grid_vel, torch.float32, 3 * N, "grid_vel"),
        _regions_ptr(region_state, polypic_region_count(grid)), _stream()),
        "polypic_grid_update_active")


def polypic_g2p(grid: polypic_grid, n_modes: int, dt: float, grid_vel: torch.Tensor,
                x_in: torch.Tensor, coeff_out: torch.Tensor,
                perm: Optional[torch.Tensor] = None, x_out: Optional[torch.Tensor] = None,
                F_in: Optional[torch.Tensor] = None, F_out: Optional[torch.Tensor] = None,
                mass_in: Optional[torch.Tensor] = None, mass_out: Optional[torch.Tensor] = None,
                status_dev: Optional[torch.Tensor] = None) -> None:
    P = x_in.numel() // 3
    N = n_nodes(grid)
    check(_lib.load().polypic_g2p(
        ctypes.byref(grid), P, int(n_modes), float(dt),
        _ptr(grid_vel, torch.float32, 3 * N, "grid_vel"),
        _ptr(x_in, torch.float32, 3 * P, "x_in"), _ptr(perm, torch.int32, P, "perm"),
        _ptr(x_out, torch.float32, 3 * P, "x_out"),
        _ptr(coeff_out, torch.float32, 3 * int(n_modes) * P, "coeff_out"),
        _ptr(F_in, torch.float32, 9 * P, "F_in"), _ptr(F_out, torch.float32, 9 * P, "F_out"),
        _ptr(mass_in, torch.float32, P, "mass_in"), _ptr(mass_out, torch.float32, P, "mass_out"),
        _ptr(status_dev, torch.int32, 1, "status_dev"), _stream()), "polypic_g2p")


def polypic_p2g_affine(grid: polypic_grid, n_modes: int, dt: float, x: torch.Tensor,
                       coeff: torch.Tensor, grid_mass: torch.Tensor, grid_mom: torch.Tensor,
                       x_fit: Optional[torch.Tensor] = None, mass: Optional[torch.Tensor] = None,
                       uniform_mass: float = 1.0, perm: Optional[torch.Tensor] = None,
                       accumulate: bool = False,
                       status_dev: Optional[torch.Tensor] = None) -> None:
    """P2G with the modes evaluated through the affine back-map of Eq. 12."""
    P = x.numel() // 3
    N = n_nodes(grid)
    check(_lib.load().polypic_p2g_affine(
        ctypes.byref(grid), P, int(n_modes), float(dt), _ptr(x, torch.float32, 3 * P, "x"),
        _ptr(x_fit, torch.float32, 3 * P, "x_fit"), _ptr(mass, torch.float32, P, "mass"),
        float(uniform_mass), _ptr(coeff, torch.float32, 3 * int(n_modes) * P, "coeff"),
        _ptr(perm, torch.int32, P, "perm"), _ptr(grid_mass, torch.float32, N, "grid_mass"),
        _ptr(grid_mom, torch.float32, 3 * N, "grid_mom"), int(bool(accumulate)),
        _ptr(status_dev, torch.int32, 1, "status_dev"), _stream()), "polypic_p2g_affine")


# ---- liquid and fabric particles on one grid: grid_mass [2][N], grid_mom / grid_vel [2][3][N]
def polypic_mixture_p2g(grid: polypic_grid, n_modes: int, x: torch.Tensor, phase: torch.Tensor,
                        mass_f: torch.Tensor, coeff: torch.Tensor, grid_mass: torch.Tensor,
                        grid_mom: torch.Tensor, mass_s: Optional[torch.Tensor] = None,
                        perm: Optional[torch.Tensor] = None, accumulate: bool = False,
                        status_dev: Optional[torch.Tensor] = None) -> None:
    P = x.numel() // 3
    N = n_nodes(grid)
    check(_lib.load().polypic_mixture_p2g(
        ctypes.byref(grid), P, int(n_modes), _ptr(x, torch.float32, 3 * P, "x"),
        _ptr(phase, torch.int32, P, "phase"), _ptr(mass_f, torch.float32, P, "mass_f"),
        _ptr(mass_s, torch.float32, P, "mass_s"),
        _ptr(coeff, torch.float32, 3 * int(n_modes) * P, "coeff"),
        _ptr(perm, torch.int32, P, "perm"), _ptr(grid_mass, torch.float32, 2 * N, "grid_mass"),
        _ptr(grid_mom, torch.float32, 6 * N, "grid_mom"), int(bool(accumulate)),
        _ptr(status_dev, torch.int32, 1, "status_dev"), _stream()), "polypic_mixture_p2g")


def polypic_mixture_grid_update(grid: polypic_grid, dt: float, gravity: Sequence[float],
                                bc_layers: int, grid_mass: torch.Tensor, grid_mom: torch.Tensor,
                                grid_vel: torch.Tensor) -> None:
    N = n_nodes(grid)
    g3 = (ctypes.c_float * 3)(*[float(v) for v in gravity])
    check(_lib.load().polypic_mixture_grid_update(
        ctypes.byref(grid), float(dt), g3, int(bc_layers),
        _ptr(grid_mass, torch.float32, 2 * N, "grid_mass"),
        _ptr(grid_mom, torch.float32, 6 * N, "grid_mom"),
        _ptr(grid_vel, torch.float32, 6 * N, "grid_vel"), _stream()),
        "polypic_mixture_grid_update")


def polypic_mixture_g2p(grid: polypic_grid, n_modes: int, dt: float, grid_vel: torch.Tensor,
                        x_in: torch.Tensor, phase_in: torch.Tensor, coeff_out: torch.Tensor,
                        perm: Optional[torch.Tensor] = None, x_out: Optional[torch.Tensor] = None,
                        F_in: Optional[torch.Tensor] = None, F_out: Optional[torch.Tensor] = None,
                        phase_out: Optional[torch.Tensor] = None,
                        mass_f_in: Optional[torch.Tensor] = None,
                        mass_f_out: Optional[torch.Tensor] = None,
                        mass_s_in: Optional[torch.Tensor] = None,
                        mass_s_out: Optional[torch.Tensor] = None,
                        status_dev: Optional[torch.Tensor] = None) -> None:
    P = x_in.numel() // 3
    N = n_nodes(grid)
    check(_lib.load().polypic_mixture_g2p(
        ctypes.byref(grid), P, int(n_modes), float(dt),
        _ptr(grid_vel, torch.float32, 6 * N, "grid_vel"),
        _ptr(x_in, torch.float32, 3 * P, "x_in"), _ptr(phase_in, torch.int32, P, "phase_in"),
        _ptr(perm, torch.int32, P, "perm"), _ptr(x_out, torch.float32, 3 * P, "x_out"),
        _ptr(coeff_out, torch.float32, 3 * int(n_modes) * P, "coeff_out"),
        _ptr(F_in, torch.float32, 9 * P, "F_in"), _ptr(F_out, torch.float32, 9 * P, "F_out"),
        _ptr(phase_out, torch.int32, P, "phase_out"),
        _ptr(mass_f_in, torch.float32, P, "mass_f_in"),
        _ptr(mass_f_out, torch.float32, P, "mass_f_out"),
        _ptr(mass_s_in, torch.float32, P, "mass_s_in"),
        _ptr(mass_s_out, torch.float32, P, "mass_s_out"),
        _ptr(status_dev, torch.int32, 1, "status_dev"), _stream()), "polypic_mixture_g2p")


# ---- staggered (MAC) grid: face arrays [3][N], component a's faces at a * N + node index
def polypic_mac_p2g(grid: polypic_grid, n_modes: int, x: torch.Tensor, coeff: torch.Tensor,
                    face_mass: torch.Tensor, face_mom: torch.Tensor,
                    mass: Optional[torch.Tensor] = None, uniform_mass: float = 1.0,
                    perm: Optional[torch.Tensor] = None, accumulate: bool = False,
                    status_dev: Optional[torch.Tensor] = None) -> None:
    P = x.numel() // 3
    N = n_nodes(grid)
    check(_lib.load().polypic_mac_p2g(
        ctypes.byref(grid), P, int(n_modes), _ptr(x, torch.float32, 3 * P, "x"),
        _ptr(mass, torch.float32, P, "mass"), float(uniform_mass),
        _ptr(coeff, torch.float32, 3 * int(n_modes) * P, "coeff"),
        _ptr(perm, torch.int32, P, "perm"),
        _ptr(face_mass, torch.float32, 3 * N, "face_mass"),
        _ptr(face_mom, torch.float32, 3 * N, "face_mom"), int(bool(accumulate)),
        _ptr(status_dev, torch.int32, 1, "status_dev"), _stream()), "polypic_mac_p2g")


def polypic_mac_grid_update(grid: polypic_grid, dt: float, gravity: Sequence[float],
                            bc_layers: int, face_mass: torch.Tensor, face_mom: torch.Tensor,
                            face_vel: torch.Tensor) -> None:
    N = n_nodes(grid)
    g3 = (ctypes.c_float * 3)(*[float(v) for v in gravity])
    check(_lib.load().polypic_mac_grid_update(
        ctypes.byref(grid), float(dt), g3, int(bc_layers),
        _ptr(face_mass, torch.float32, 3 * N, "face_mass"),
        _ptr(face_mom, torch.float32, 3 * N, "face_mom"),
        _ptr(face_vel, torch.float32, 3 * N, "face_vel"), _stream()), "polypic_mac_grid_update")


def polypic_mac_g2p(grid: polypic_grid, n_modes: int, dt: float, face_vel: torch.Tensor,
                    x_in: torch.Tensor, coeff_out: torch.Tensor,
                    perm: Optional[torch.Tensor] = None, x_out: Optional[torch.Tensor] = None,
                    F_in: Optional[torch.Tensor] = None, F_out: Optional[torch.Tensor] = None,
                    mass_in: Optional[torch.Tensor] = None,
                    mass_out: Optional[torch.Tensor] = None,
                    status_dev: Optional[torch.Tensor] = None) -> None:
    P = x_in.numel() // 3
    N = n_nodes(grid)
    check(_lib.load().polypic_mac_g2p(
        ctypes.byref(grid), P, int(n_modes), float(dt),
        _ptr(face_vel, torch.float32, 3 * N, "face_vel"),
        _ptr(x_in, torch.float32, 3 * P, "x_in"), _ptr(perm, torch.int32, P, "perm"),
        _ptr(x_out, torch.float32, 3 * P, "x_out"),
        _ptr(coeff_out, torch.float32, 3 * int(n_modes) * P, "coeff_out"),
        _ptr(F_in, torch.float32, 9 * P, "F_in"), _ptr(F_out, torch.float32, 9 * P, "F_out"),
        _ptr(mass_in, torch.float32, P, "mass_in"), _ptr(mass_out, torch.float32, P, "mass_out"),
        _ptr(status_dev, torch.int32, 1, "status_dev"), _stream()), "polypic_mac_g2p")


def polypic_g2p2g(grid: polypic_grid, n_modes: int, dt: float, grid_vel: torch.Tensor,
                  x_in: torch.Tensor, x_out: torch.Tensor, coeff_out: torch.Tensor,
                  grid_mass: torch.Tensor, grid_mom: torch.Tensor,
                  perm: Optional[torch.Tensor] = None,
                  F_in: Optional[torch.Tensor] = None, F_out: Optional[torch.Tensor] = None,
                  mass_in: Optional[torch.Tensor] = None, mass_out: Optional[torch.Tensor] = None,
                  uniform_mass: float = 1.0,
                  status_dev: Optional[torch.Tensor] = None, accumulate: bool = False,
                  region_state: Optional[torch.Tensor] = None) -> None:
    """accumulate: add to grid_mass / grid_mom instead of clearing them first;
    region_state: flag the regions the scatter lands in."""
    P = x_in.numel() // 3
    N = n_nodes(grid)
    check(_lib.load().polypic_g2p2g(
        ctypes.byref(grid), P, int(n_modes), float(dt),
        _ptr(grid_vel, torch.float32, 3 * N, "grid_vel"),
        _ptr(x_in, torch.float32, 3 * P, "x_in"), _ptr(perm, torch.int32, P, "perm"),
        _ptr(x_out, torch.float32, 3 * P, "x_out"),
        _ptr(coeff_out, torch.float32, 3 * int(n_modes) * P, "coeff_out"),
        _ptr(F_in, torch.float32, 9 * P, "F_in"), _ptr(F_out, torch.float32, 9 * P, "F_out"),
        _ptr(mass_in, torch.float32, P, "mass_in"), _ptr(mass_out, torch.float32, P, "mass_out"),
        float(uniform_mass),
        _ptr(grid_mass, torch.float32, N, "grid_mass"),
        _ptr(grid_mom, torch.float32, 3 * N, "grid_mom"), int(bool(accumulate)),
        _regions_ptr(region_state, polypic_region_count(grid)),
        _ptr(status_dev, torch.int32, 1, "status_dev"), _stream()), "polypic_g2p2g")


class FusedChoice(NamedTuple):
    """Launch choice of polypic_g2p2g: lane-group size and chunk order (POLYPIC_SCHED_*)."""

    lane_group: int
    schedule: int


def polypic_set_g2p2g_config(n_modes: int, lane_group: int = -1, schedule: int = -1) -> None:
    """Lane-group size (2 or 4) and chunk order (POLYPIC_SCHED_LINEAR or _XCD) of
    polypic_g2p2g at this mode count; -1 for a default."""
    check(_lib.load().polypic_set_g2p2g_config(int(n_modes), int(lane_group), int(schedule)),
          "polypic_set_g2p2g_config")


def polypic_get_g2p2g_config(n_modes: int) -> FusedChoice:
    lg, sc = ctypes.c_int32(0), ctypes.c_int32(0)
    check(_lib.load().polypic_get_g2p2g_config(int(n_modes), ctypes.byref(lg), ctypes.byref(sc)),
          "polypic_get_g2p2g_config")
    return FusedChoice(int(lg.value), int(sc.value))


def polypic_autotune_g2p2g(grid: polypic_grid, n_modes: int, dt: float, grid_vel: torch.Tensor,
                           x_in: torch.Tensor, x_out: torch.Tensor, coeff_out: torch.Tensor,
                           grid_mass: torch.Tensor, grid_mom: torch.Tensor,
                           perm: Optional[torch.Tensor] = None,
                           F_in: Optional[torch.Tensor] = None,
                           F_out: Optional[torch.Tensor] = None,
                           mass_in: Optional[torch.Tensor] = None,
                           mass_out: Optional[torch.Tensor] = None,
                           uniform_mass: float = 1.0) -> FusedChoice:
    """Times polypic_g2p2g with lane groups of 2 and 4, in launch and in XCD chunk order, on
    these arguments (synchronises), keeps the fastest for this mode count and returns it;
    the outputs are the call's."""
    P = x_in.numel() // 3
    N = n_nodes(grid)
    out, sched = ctypes.c_int32(0), ctypes.c_int32(0)
    check(_lib.load().polypic_autotune_g2p2g(
        ctypes.byref(grid), P, int(n_modes), float(dt),
        _ptr(grid_vel, torch.float32, 3 * N, "grid_vel"),
        _ptr(x_in, torch.float32, 3 * P, "x_in"), _ptr(perm, torch.int32, P, "perm"),
        _ptr(x_out, torch.float32, 3 * P, "x_out"),
        _ptr(coeff_out, torch.float32, 3 * int(n_modes) * P, "coeff_out"),
        _ptr(F_in, torch.float32, 9 * P, "F_in"), _ptr(F_out, torch.float32, 9 * P, "F_out"),
        _ptr(mass_in, torch.float32, P, "mass_in"), _ptr(mass_out, torch.float32, P, "mass_out"),
        float(uniform_mass),
        _ptr(grid_mass, torch.float32, N, "grid_mass"),
        _ptr(grid_mom, torch.float32, 3 * N, "grid_mom"), ctypes.byref(out),
        ctypes.byref(sched), _stream()), "polypic_autotune_g2p2g")
    return FusedChoice(int(out.value), int(sched.value))


def polypic_g2p_backward(grid: polypic_grid, n_modes: int, dt: float, grid_vel: torch.Tensor,
                         x_in: torch.Tensor, coeff_out_grad: torch.Tensor,
                         grid_vel_grad: torch.Tensor, x_in_grad: torch.Tensor,
                         perm: Optional[torch.Tensor] = None,
                         x_out_grad: Optional[torch.Tensor] = None, accumulate: bool = False,
                         status_dev: Optional[torch.Tensor] = None) -> None:
    P = x_in.numel() // 3
    N = n_nodes(grid)
    check(_lib.load().polypic_g2p_backward(
        ctypes.byref(grid), P, int(n_modes), float(dt),
        _ptr(grid_vel, torch.float32, 3 * N, "grid_vel"),
        _ptr(x_in, torch.float32, 3 * P, "x_in"), _ptr(perm, torch.int32, P, "perm"),
        _ptr(coeff_out_grad, torch.float32, 3 * int(n_modes) * P, "coeff_out_grad"),
        _ptr(x_out_grad, torch.float32, 3 * P, "x_out_grad"),
        _ptr(grid_vel_grad, torch.float32, 3 * N, "grid_vel_grad"), int(bool(accumulate)),
        _ptr(x_in_grad, torch.float32, 3 * P, "x_in_grad"),
        _ptr(status_dev, torch.int32, 1, "status_dev"), _stream()), "polypic_g2p_backward")


def polypic_grid_update_backward(grid: polypic_grid, dt: float, gravity: Sequence[float],
                                 bc_layers: int, grid_mass: torch.Tensor, grid_mom: torch.Tensor,
                                 grid_vel_grad: torch.Tensor, grid_mass_grad: torch.Tensor,
                                 grid_mom_grad: torch.Tensor) -> None:
    N = n_nodes(grid)
    g3 = (ctypes.c_float * 3)(*[float(v) for v in gravity])
    check(_lib.load().polypic_grid_update_backward(
        ctypes.byref(grid), float(dt), g3, int(bc_layers),
        _ptr(grid_mass, torch.float32, N, "grid_mass"),
        _ptr(grid_mom, torch.float32, 3 * N, "grid_mom"),
        _ptr(grid_vel_grad, torch.float32, 3 * N, "grid_vel_grad"),
        _ptr(grid_mass_grad, torch.float32, N, "grid_mass_grad"),
        _ptr(grid_mom_grad, torch.float32, 3 * N, "grid_mom_grad"), _stream()),
        "polypic_grid_update_backward")


def polypic_p2g_backward(grid: polypic_grid, n_modes: int, x: torch.Tensor, coeff: torch.Tensor,
                         grid_mass_grad: torch.Tensor, grid_mom_grad: torch.Tensor,
                         coeff_grad: torch.Tensor, x_grad: torch.Tensor,
                         mass: Optional[torch.Tensor] = None, uniform_mass: float = 1.0,
                         perm: Optional[torch.Tensor] = None,
                         mass_grad: Optional[torch.Tensor] = None,
                         status_dev: Optional[torch.Tensor] = None) -> None:
    P = x.numel() // 3
    N = n_nodes(grid)
    check(_lib.load().polypic_p2g_backward(
        ctypes.byref(grid), P, int(n_modes), _ptr(x, torch.float32, 3 * P, "x"),
        _ptr(mass, torch.float32, P, "mass"), float(uniform_mass),
        _ptr(coeff, torch.float32, 3 * int(n_modes) * P, "coeff"),
        _ptr(perm, torch.int32, P, "perm"),
        _ptr(grid_mass_grad, torch.float32, N, "grid_mass_grad"),
        _ptr(grid_mom_grad, torch.float32, 3 * N, "grid_mom_grad"),
        _ptr(coeff_grad, torch.float32, 3 * int(n_modes) * P, "coeff_grad"),
        _ptr(x_grad, torch.float32, 3 * P, "x_grad"), _ptr(mass_grad, torch.float32, P, "mass_grad"),
        _ptr(status_dev, torch.int32, 1, "status_dev"), _stream()), "polypic_p2g_backward")


# ---------------------------------------------------------------- particle order
def _rows_call(name: str, src: torch.Tensor, dst: torch.Tensor, idx: torch.Tensor) -> None:
    if src.dtype not in (torch.float32, torch.int32):
        raise TypeError(f"src must be float32 or int32, got {src.dtype}")
    if dst.dtype != src.dtype or dst.shape != src.shape:
        raise ValueError("dst must have the dtype and shape of src")
    P = src.shape[-1] if src.dim() > 0 else 0
    rows = src.numel() // P if P else 0
    check(getattr(_lib.load(), name)(
        _ptr(src, src.dtype, rows * P, "src"), _ptr(dst, src.dtype, rows * P, "dst"),
        _ptr(idx, torch.int32, P, "idx"), rows, P, _stream()), name)


def polypic_gather_rows(src: torch.Tensor, dst: torch.Tensor, idx: torch.Tensor) -> None:
    """dst[..., i] = src[..., idx[i]] over the last axis (P), for float32 or int32 arrays of
    the same shape; idx is an int32 array of P indices."""
    _rows_call("polypic_gather_rows", src, dst, idx)


def polypic_scatter_rows(src: torch.Tensor, dst: torch.Tensor, idx: torch.Tensor) -> None:
    """dst[..., idx[i]] = src[..., i] over the last axis (P), as polypic_gather_rows."""
    _rows_call("polypic_scatter_rows", src, dst, idx)


def polypic_invert_permutation(perm: torch.Tensor, inv: torch.Tensor) -> None:
    """inv[perm[i]] = i for an int32 permutation of [0, P)."""
    P = perm.numel()
    check(_lib.load().polypic_invert_permutation(
        _ptr(perm, torch.int32, P, "perm"), _ptr(inv, torch.int32, P, "inv"), P, _stream()),
        "polypic_invert_permutation")


# ---------------------------------------------------------------- batches
class Batch:
    """A planned batch of scenes: the sealed C descriptor plus the device table it points to.

    scenes: list of (polypic_grid, n_particles).  Particles of scene k occupy the
    flattened range [p_offset_k, p_offset_k + n_k) in scene order; its nodes the
    range [node_offset_k, node_offset_k + nodes_k), scenes packed end to end.
    """

    def __init__(self, scenes: Sequence[Tuple[polypic_grid, int]], device="cuda"):
        lib = _lib.load()
        n = len(scenes)
        arr = (_lib.polypic_scene * n)()
        p = 0
        node = 0
        self.p_offsets: List[int] = []
        self.node_offsets: List[int] = []
        self.grids: List[polypic_grid] = []
        for k, (g, count) in enumerate(scenes):
            arr[k].grid = g
            arr[k].p_offset = p
            arr[k].n_particles = int(count)
            arr[k].node_offset = node
            self.p_offsets.append(p)
            self.node_offsets.append(node)
            self.grids.append(g)
            p += int(count)
            node += n_nodes(g)
        self.p_offsets.append(p)
        self.node_offsets.append(node)
        nbytes = ctypes.c_size_t(0)
        check(lib.polypic_batch_table_bytes(n, ctypes.byref(nbytes)), "polypic_batch_table_bytes")
        self.table = torch.empty(max(1, nbytes.value), dtype=torch.uint8, device=device)
        self.desc = _lib.polypic_batch()
        check(lib.polypic_batch_plan(arr, n, node, ctypes.c_void_p(self.table.data_ptr()),
                                     self.table.numel(), ctypes.byref(self.desc), _stream()),
              "polypic_batch_plan")
        self.P = int(self.desc.P)
        self.N = int(self.desc.N)
        self.n_regions = int(self.desc.n_regions)
        self.n_scenes = n

    def ref(self):
        return ctypes.byref(self.desc)


def polypic_batch_sort_workspace_bytes(batch: Batch) -> int:
    out = ctypes.c_size_t(0)
    check(_lib.load().polypic_batch_sort_workspace_bytes(batch.ref(), ctypes.byref(out)),
          "polypic_batch_sort_workspace_bytes")
    return int(out.value)


def polypic_batch_sort(batch: Batch, x: torch.Tensor, keys_out: torch.Tensor,
                       perm_out: torch.Tensor, ws: torch.Tensor,
                       status_dev: Optional[torch.Tensor] = None) -> None:
    P = batch.P
    check(_lib.load().polypic_batch_sort(
        batch.ref(), _ptr(x, torch.float32, 3 * P, "x"), _keys_ptr(keys_out, P),
        _ptr(perm_out, torch.int32, P, "perm_out"), _ptr(ws, torch.uint8, ws.numel(), "ws"),
        ws.numel(), _ptr(status_dev, torch.int32, 1, "status_dev"), _stream()), "polypic_batch_sort")


def polypic_batch_sort_update_workspace_bytes(batch: Batch) -> int:
    out = ctypes.c_size_t(0)
    check(_lib.load().polypic_batch_sort_update_workspace_bytes(batch.ref(), ctypes.byref(out)),
          "polypic_batch_sort_update_workspace_bytes")
    return int(out.value)


def polypic_batch_sort_update(batch: Batch, x: torch.Tensor, keys_prev: torch.Tensor,
                              keys_out: torch.Tensor, perm_out: torch.Tensor, ws: torch.Tensor,
                              status_dev: Optional[torch.Tensor] = None) -> None:
    P = batch.P
    check(_lib.load().polypic_batch_sort_update(
        batch.ref(), _ptr(x, torch.float32, 3 * P, "x"), _keys_ptr(keys_prev, P),
        _keys_ptr(keys_out, P), _ptr(perm_out, torch.int32, P, "perm_out"),
        _ptr(ws, torch.uint8, ws.numel(), "ws"), ws.numel(),
        _ptr(status_dev, torch.int32, 1, "status_dev"), _stream()), "polypic_batch_sort_update")


def polypic_batch_p2g(batch: Batch, n_modes: int, x: torch.Tensor, coeff: torch.Tensor,
                      grid_mass: torch.Tensor, grid_mom: torch.Tensor,
                      mass: Optional[torch.Tensor] = None, uniform_mass: float = 1.0,
                      perm: Optional[torch.Tensor] = None, accumulate: bool = False,
                      status_dev: Optional[torch.Tensor] = None) -> None:
    P, N = batch.P, batch.N
    check(_lib.load().polypic_batch_p2g(
        batch.ref(), int(n_modes), _ptr(x, torch.float32, 3 * P, "x"),
        _ptr(mass, torch.float32, P, "mass"), float(uniform_mass),
        _ptr(coeff, torch.float32, 3 * int(n_modes) * P, "coeff"),
        _ptr(perm, torch.int32, P, "perm"), _ptr(grid_mass, torch.float32, N, "grid_mass"),
        _ptr(grid_mom, torch.float32, 3 * N, "grid_mom"), int(bool(accumulate)),
        _ptr(status_dev, torch.int32, 1, "status_dev"), _stream()), "polypic_batch_p2g")


def polypic_batch_grid_update(batch: Batch, dt: float, gravity: Sequence[float], bc_layers: int,
                              grid_mass: torch.Tensor, grid_mom: torch.Tensor,
                              grid_vel: torch.Tensor) -> None:
    N = batch.N
    g3 = (ctypes.c_float * 3)(*[float(v) for v in gravity])
    check(_lib.load().polypic_batch_grid_update(
        batch.ref(), float(dt), g3, int(bc_layers),
        _ptr(grid_mass, torch.float32, N, "grid_mass"),
        _ptr(grid_mom, torch.float32, 3 * N, "grid_mom"),
        _ptr(grid_vel, torch.float32, 3 * N, "grid_vel"), _stream()), "polypic_batch_grid_update")


def polypic_batch_g2p(batch: Batch, n_modes: int, dt: float, grid_vel: torch.Tensor,
                      x_in: torch.Tensor, coeff_out: torch.Tensor,
                      perm: Optional[torch.Tensor] = None, x_out: Optional[torch.Tensor] = None,
                      F_in: Optional[torch.Tensor] = None, F_out: Optional[torch.Tensor] = None,
                      mass_in: Optional[torch.Tensor] = None,
                      mass_out: Optional[torch.Tensor] = None,
                      status_dev: Optional[torch.Tensor] = None) -> None:
    P, N = batch.P, batch.N
    check(_lib.load().polypic_batch_g2p(
        batch.ref(), int(n_modes), float(dt), _ptr(grid_vel, torch.float32, 3 * N, "grid_vel"),
        _ptr(x_in, torch.float32, 3 * P, "x_in"), _ptr(perm, torch.int32, P, "perm"),
        _ptr(x_out, torch.float32, 3 * P, "x_out"),
        _ptr(coeff_out, torch.float32, 3 * int(n_modes) * P, "coeff_out"),
        _ptr(F_in, torch.float32, 9 * P, "F_in"), _ptr(F_out, torch.float32, 9 * P, "F_out"),
        _ptr(mass_in, torch.float32, P, "mass_in"), _ptr(mass_out, torch.float32, P, "mass_out"),
        _ptr(status_dev, torch.int32, 1, "status_dev"), _stream()), "polypic_batch_g2p")


def polypic_batch_g2p2g(batch: Batch, n_modes: int, dt: float, grid_vel: torch.Tensor,
                        x_in: torch.Tensor, x_out: torch.Tensor, coeff_out: torch.Tensor,
                        grid_mass: torch.Tensor, grid_mom: torch.Tensor,
                        perm: Optional[torch.Tensor] = None,
                        F_in: Optional[torch.Tensor] = None, F_out: Optional[torch.Tensor] = None,
                        mass_in: Optional[torch.Tensor] = None,
                        mass_out: Optional[torch.Tensor] = None, uniform_mass: float = 1.0,
                        status_dev: Optional[torch.Tensor] = None, accumulate: bool = False,
                        region_state: Optional[torch.Tensor] = None) -> None:
    P, N = batch.P, batch.N
    check(_lib.load().polypic_batch_g2p2g(
        batch.ref(), int(n_modes), float(dt), _ptr(grid_vel, torch.float32, 3 * N, "grid_vel"),
        _ptr(x_in, torch.float32, 3 * P, "x_in"), _ptr(perm, torch.int32, P, "perm"),
        _ptr(x_out, torch.float32, 3 * P, "x_out"),
        _ptr(coeff_out, torch.float32, 3 * int(n_modes) * P, "coeff_out"),
        _ptr(F_in, torch.float32, 9 * P, "F_in"), _ptr(F_out, torch.float32, 9 * P, "F_out"),
        _ptr(mass_in, torch.float32, P, "mass_in"), _ptr(mass_out, torch.float32, P, "mass_out"),
        float(uniform_mass), _ptr(grid_mass, torch.float32, N, "grid_mass"),
        _ptr(grid_mom, torch.float32, 3 * N, "grid_mom"), int(bool(accumulate)),
        _regions_ptr(region_state, batch.n_regions),
        _ptr(status_dev, torch.int32, 1, "status_dev"), _stream()), "polypic_batch_g2p2g")


def polypic_batch_grid_update_active(batch: Batch, dt: float, gravity: Sequence[float],
                                     bc_layers: int, grid_mass: torch.Tensor,
                                     grid_mom: torch.Tensor, grid_vel: torch.Tensor,
                                     region_state: torch.Tensor) -> None:
    N = batch.N
    g3 = (ctypes.c_float * 3)(*[float(v) for v in gravity])
    check(_lib.load().polypic_batch_grid_update_active(
        batch.ref(), float(dt), g3, int(bc_layers),
        _ptr(grid_mass, torch.float32, N, "grid_mass"),
        _ptr(grid_mom, torch.float32, 3 * N, "grid_mom"),
        _ptr(grid_vel, torch.float32, 3 * N, "grid_vel"),
        _regions_ptr(region_state, batch.n_regions), _stream()),
        "polypic_batch_grid_update_active")


class BatchChoice(NamedTuple):
    """Batched P2G launch configuration: workgroup size, chunk schedule, persistent
    workgroups per CU, brick edge in cells."""

    block: int
    schedule: int
    per_cu: int = 0
    brick: int = 4


def polypic_batch_set_config(n_modes: int, block: int, schedule: int, per_cu: int = 0,
                             brick: int = 4) -> None:
    check(_lib.load().polypic_batch_set_config(int(n_modes), int(block), int(schedule),
                                               int(per_cu), int(brick)),
          "polypic_batch_set_config")


def polypic_batch_get_config(n_modes: int) -> BatchChoice:
    v = [ctypes.c_int32(0) for _ in range(4)]
    check(_lib.load().polypic_batch_get_config(int(n_modes), *[ctypes.byref(t) for t in v]),
          "polypic_batch_get_config")
    return BatchChoice(*(int(t.value) for t in v))


def polypic_batch_autotune(batch: Batch, n_modes: int, x: torch.Tensor, coeff: torch.Tensor,
                           grid_mass: torch.Tensor, grid_mom: torch.Tensor,
                           mass: Optional[torch.Tensor] = None, uniform_mass: float = 1.0,
                           perm: Optional[torch.Tensor] = None) -> BatchChoice:
    P, N = batch.P, batch.N
    v = [ctypes.c_int32(0) for _ in range(4)]
    check(_lib.load().polypic_batch_autotune(
        batch.ref(), int(n_modes), _ptr(x, torch.float32, 3 * P, "x"),
        _ptr(mass, torch.float32, P, "mass"), float(uniform_mass),
        _ptr(coeff, torch.float32, 3 * int(n_modes) * P, "coeff"),
        _ptr(perm, torch.int32, P, "perm"), _ptr(grid_mass, torch.float32, N, "grid_mass"),
        _ptr(grid_mom, torch.float32, 3 * N, "grid_mom"), *[ctypes.byref(t) for t in v],
        _stream()), "polypic_batch_autotune")
    return BatchChoice(*(int(t.value) for t in v))
