"""ctypes loader for libpolypic.so and the C declarations of its entry points.

The library must have been built (``python -m paper_2308_01060_amd.build`` or
``__graft_entry__.build()``); importing this module without it raises, so no
caller can run without the HIP code.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpolypic.so")

POLYPIC_OK = 0
POLYPIC_EINVAL = 1
POLYPIC_ERANGE = 2
POLYPIC_EDEVICE = 3
POLYPIC_ENOSPACE = 4
POLYPIC_ENOTSUP = 5
POLYPIC_FLAG_RANGE = 1
POLYPIC_FLAG_ORDER = 2
POLYPIC_FLAG_STALL = 4
POLYPIC_FLAG_PHASE = 8
POLYPIC_FLAG_MAP = 16
POLYPIC_SORT_NOALLOC_MAX_P = 2097152
POLYPIC_P2G_DEFAULT = -1
POLYPIC_P2G_BRICKS = 0
POLYPIC_P2G_CELLS = 1
POLYPIC_SCHED_LINEAR = 0
POLYPIC_SCHED_XCD = 1
POLYPIC_SCHED_PERSISTENT = 2

EXPORTED = (
    "polypic_strerror",
    "polypic_version",
    "polypic_last_device_error",
    "polypic_sort_workspace_bytes",
    "polypic_sort",
    "polypic_sort_noalloc",
    "polypic_sort_update_workspace_bytes",
    "polypic_sort_update",
    "polypic_p2g_workspace_bytes",
    "polypic_p2g",
    "polypic_set_p2g_config",
    "polypic_get_p2g_config",
    "polypic_autotune_p2g",
    "polypic_set_g2p_schedule",
    "polypic_get_g2p_schedule",
    "polypic_grid_update",
    "polypic_grid_update_clear",
    "polypic_region_count",
    "polypic_grid_update_active",
    "polypic_g2p",
    "polypic_g2p2g",
    "polypic_set_g2p2g_config",
    "polypic_get_g2p2g_config",
    "polypic_autotune_g2p2g",
    "polypic_p2g_affine",
    "polypic_mixture_p2g",
    "polypic_mixture_grid_update",
    "polypic_mixture_g2p",
    "polypic_mac_p2g",
    "polypic_mac_grid_update",
    "polypic_mac_g2p",
    "polypic_g2p_backward",
    "polypic_grid_update_backward",
    "polypic_p2g_backward",
    "polypic_gather_rows",
    "polypic_scatter_rows",
    "polypic_invert_permutation",
    "polypic_batch_table_bytes",
    "polypic_batch_plan",
    "polypic_batch_sort_workspace_bytes",
    "polypic_batch_sort",
    "polypic_batch_sort_update_workspace_bytes",
    "polypic_batch_sort_update",
    "polypic_batch_p2g",
    "polypic_batch_grid_update",
    "polypic_batch_g2p",
    "polypic_batch_g2p2g",
    "polypic_batch_grid_update_active",
    "polypic_batch_set_config",
    "polypic_batch_get_config",
    "polypic_batch_autotune",
)


class polypic_grid(ctypes.Structure):
    """Mirror of ``struct polypic_grid`` (include/polypic.h)."""

    _fields_ = [
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("nz", ctypes.c_int32),
        ("dx", ctypes.c_float),
        ("inv_dx", ctypes.c_float),
        ("origin", ctypes.c_float * 3),
    ]


class polypic_scene(ctypes.Structure):
    """Mirror of ``struct polypic_scene``."""

    _fields_ = [
        ("grid", polypic_grid),
        ("p_offset", ctypes.c_int64),
        ("n_particles", ctypes.c_int64),
        ("node_offset", ctypes.c_int64),
    ]


class polypic_batch(ctypes.Structure):
    """Mirror of ``struct polypic_batch`` (filled by polypic_batch_plan)."""

    _fields_ = [
        ("n_scenes", ctypes.c_int32),
        ("key_bits", ctypes.c_int32),
        ("morton_bits", ctypes.c_int32),
        ("max_nodes", ctypes.c_int32),
        ("P", ctypes.c_int64),
        ("N", ctypes.c_int64),
        ("n_regions", ctypes.c_int64),
        ("table", ctypes.c_void_p),
        ("seal", ctypes.c_uint64),
    ]


class PolyPICError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        detail = ""
        if code == POLYPIC_EDEVICE:
            detail = " [" + load().polypic_last_device_error().decode() + "]"
        super().__init__(f"{where}: {strerror(code)} (status {code}){detail}")


_lib = None


def load() -> ctypes.CDLL:
    """Load libpolypic.so once and declare the signatures; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python paper_2308_01060_amd/build.py)")
    # torch ships its own HIP runtime under the same soname (libamdhip64.so.7).
    # Loading torch first makes libpolypic.so bind to that runtime, so the
    # library and torch share one HIP context, its devices, memory and streams.
    # Loaded the other way round, the process would hold two HIP runtimes and
    # the library's would see no device.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32, i64, f32, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_size_t
    G = ctypes.POINTER(polypic_grid)
    lib.polypic_strerror.restype = ctypes.c_char_p
    lib.polypic_strerror.argtypes = [i32]
    lib.polypic_version.restype = i32
    lib.polypic_version.argtypes = []
    lib.polypic_last_device_error.restype = ctypes.c_char_p
    lib.polypic_last_device_error.argtypes = []
    lib.polypic_sort_workspace_bytes.restype = i32
    lib.polypic_sort_workspace_bytes.argtypes = [G, i64, ctypes.POINTER(sz)]
    lib.polypic_sort.restype = i32
    lib.polypic_sort.argtypes = [G, i64, P, P, P, P, sz, P, P]
    lib.polypic_sort_noalloc.restype = i32
    lib.polypic_sort_noalloc.argtypes = [G, i64, P, P, P, P, P]
    lib.polypic_sort_update_workspace_bytes.restype = i32
    lib.polypic_sort_update_workspace_bytes.argtypes = [G, i64, ctypes.POINTER(sz)]
    lib.polypic_sort_update.restype = i32
    lib.polypic_sort_update.argtypes = [G, i64, P, P, P, P, P, sz, P, P]
    lib.polypic_p2g_workspace_bytes.restype = i32
    lib.polypic_p2g_workspace_bytes.argtypes = [G, i64, ctypes.POINTER(sz)]
    lib.polypic_p2g.restype = i32
    lib.polypic_p2g.argtypes = [G, i64, i32, P, P, f32, P, P, P, P, sz, P, P, i32, P, P]
    lib.polypic_set_p2g_config.restype = i32
    lib.polypic_set_p2g_config.argtypes = [i32, i32, i32, i32, i32, i32]
    pi = ctypes.POINTER(i32)
    lib.polypic_get_p2g_config.restype = i32
    lib.polypic_get_p2g_config.argtypes = [i32, pi, pi, pi, pi, pi]
    lib.polypic_autotune_p2g.restype = i32
    lib.polypic_autotune_p2g.argtypes = [G, i64, i32, P, P, f32, P, P, P, P, sz, P, P,
                                         pi, pi, pi, pi, pi, P]
    lib.polypic_set_g2p_schedule.restype = i32
    lib.polypic_set_g2p_schedule.argtypes = [i32]
    lib.polypic_get_g2p_schedule.restype = i32
    lib.polypic_get_g2p_schedule.argtypes = [pi]
    lib.polypic_grid_update.restype = i32
    lib.polypic_grid_update.argtypes = [G, f32, ctypes.POINTER(f32), i32, P, P, P, P]
    lib.polypic_grid_update_clear.restype = i32
    lib.polypic_grid_update_clear.argtypes = [G, f32, ctypes.POINTER(f32), i32, P, P, P, P]
    lib.polypic_region_count.restype = i32
    lib.polypic_region_count.argtypes = [G, ctypes.POINTER(i64)]
    lib.polypic_grid_update_active.restype = i32
    lib.polypic_grid_update_active.argtypes = [G, f32, ctypes.POINTER(f32), i32, P, P, P, P, P]
    lib.polypic_g2p.restype = i32
    lib.polypic_g2p.argtypes = [G, i64, i32, f32, P, P, P, P, P, P, P, P, P, P, P]
    lib.polypic_mixture_p2g.restype = i32
    lib.polypic_mixture_p2g.argtypes = [G, i64, i32, P, P, P, P, P, P, P, P, i32, P, P]
    lib.polypic_mixture_grid_update.restype = i32
    lib.polypic_mixture_grid_update.argtypes = [G, f32, ctypes.POINTER(f32), i32, P, P, P, P]
    lib.polypic_mixture_g2p.restype = i32
    lib.polypic_mixture_g2p.argtypes = [G, i64, i32, f32, P, P, P, P, P, P, P, P, P, P, P, P,
                                        P, P, P]
    lib.polypic_p2g_affine.restype = i32
    lib.polypic_p2g_affine.argtypes = [G, i64, i32, f32, P, P, P, f32, P, P, P, P, i32, P, P]
    lib.polypic_mac_p2g.restype = i32
    lib.polypic_mac_p2g.argtypes = [G, i64, i32, P, P, f32, P, P, P, P, i32, P, P]
    lib.polypic_mac_grid_update.restype = i32
    lib.polypic_mac_grid_update.argtypes = [G, f32, ctypes.POINTER(f32), i32, P, P, P, P]
    lib.polypic_mac_g2p.restype = i32
    lib.polypic_mac_g2p.argtypes = [G, i64, i32, f32, P, P, P, P, P, P, P, P, P, P, P]
    lib.polypic_g2p2g.restype = i32
    lib.polypic_g2p2g.argtypes = [G, i64, i32, f32, P, P, P, P, P, P, P, P, P, f32, P, P, i32,
                                  P, P, P]
    lib.polypic_set_g2p2g_config.restype = i32
    lib.polypic_set_g2p2g_config.argtypes = [i32, i32, i32]
    lib.polypic_get_g2p2g_config.restype = i32
    lib.polypic_get_g2p2g_config.argtypes = [i32, pi, pi]
    lib.polypic_autotune_g2p2g.restype = i32
    lib.polypic_autotune_g2p2g.argtypes = [G, i64, i32, f32, P, P, P, P, P, P, P, P, P, f32, P,
                                           P, pi, pi, P]
    lib.polypic_g2p_backward.restype = i32
    lib.polypic_g2p_backward.argtypes = [G, i64, i32, f32, P, P, P, P, P, P, i32, P, P, P]
    lib.polypic_grid_update_backward.restype = i32
    lib.polypic_grid_update_backward.argtypes = [G, f32, ctypes.POINTER(f32), i32, P, P, P, P, P,
                                                 P]
    lib.polypic_p2g_backward.restype = i32
    lib.polypic_p2g_backward.argtypes = [G, i64, i32, P, P, f32, P, P, P, P, P, P, P, P, P]
    lib.polypic_gather_rows.restype = i32
    lib.polypic_gather_rows.argtypes = [P, P, P, i64, i64, P]
    lib.polypic_scatter_rows.restype = i32
    lib.polypic_scatter_rows.argtypes = [P, P, P, i64, i64, P]
    lib.polypic_invert_permutation.restype = i32
    lib.polypic_invert_permutation.argtypes = [P, P, i64, P]
    B = ctypes.POINTER(polypic_batch)
    lib.polypic_batch_table_bytes.restype = i32
    lib.polypic_batch_table_bytes.argtypes = [i32, ctypes.POINTER(sz)]
    lib.polypic_batch_plan.restype = i32
    lib.polypic_batch_plan.argtypes = [ctypes.POINTER(polypic_scene), i32, i64, P, sz, B, P]
    lib.polypic_batch_sort_workspace_bytes.restype = i32
    lib.polypic_batch_sort_workspace_bytes.argtypes = [B, ctypes.POINTER(sz)]
    lib.polypic_batch_sort.restype = i32
    lib.polypic_batch_sort.argtypes = [B, P, P, P, P, sz, P, P]
    lib.polypic_batch_sort_update_workspace_bytes.restype = i32
    lib.polypic_batch_sort_update_workspace_bytes.argtypes = [B, ctypes.POINTER(sz)]
    lib.polypic_batch_sort_update.restype = i32
    lib.polypic_batch_sort_update.argtypes = [B, P, P, P, P, P, sz, P, P]
    lib.polypic_batch_p2g.restype = i32
    lib.polypic_batch_p2g.argtypes = [B, i32, P, P, f32, P, P, P, P, i32, P, P]
    lib.polypic_batch_grid_update.restype = i32
    lib.polypic_batch_grid_update.argtypes = [B, f32, ctypes.POINTER(f32), i32, P, P, P, P]
    lib.polypic_batch_g2p.restype = i32
    lib.polypic_batch_g2p.argtypes = [B, i32, f32, P, P, P, P, P, P, P, P, P, P, P]
    lib.polypic_batch_g2p2g.restype = i32
    lib.polypic_batch_g2p2g.argtypes = [B, i32, f32, P, P, P, P, P, P, P, P, P, f32, P, P, i32, P,
                                        P, P]
    lib.polypic_batch_grid_update_active.restype = i32
    lib.polypic_batch_grid_update_active.argtypes = [B, f32, ctypes.POINTER(f32), i32, P, P, P,
                                                     P, P]
    lib.polypic_batch_set_config.restype = i32
    lib.polypic_batch_set_config.argtypes = [i32, i32, i32, i32, i32]
    lib.polypic_batch_get_config.restype = i32
    lib.polypic_batch_get_config.argtypes = [i32, pi, pi, pi, pi]
    lib.polypic_batch_autotune.restype = i32
    lib.polypic_batch_autotune.argtypes = [B, i32, P, P, f32, P, P, P, P, pi, pi, pi, pi, P]
    _lib = lib
    return lib


def strerror(code: int) -> str:
    return load().polypic_strerror(int(code)).decode()


def check(code: int, where: str) -> None:
    if code != POLYPIC_OK:
        raise PolyPICError(code, where)
