"""Helpers for the GPU parity tests: move seeded inputs to the device, run the
library through the C ABI, and compare with the FP64 oracle."""
from __future__ import annotations

import contextlib
import sys

import numpy as np
import pytest
import torch

from oracle import polypic_oracle as O

# Parity bar (normwise relative error, FP32 device vs FP64 oracle) on grid mass,
# grid momentum and particle coefficients.
TOL_NORMWISE = 1e-5


def require_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    import paper_2308_01060_amd as pp  # noqa: F401  (fails loudly without the HIP library)
    return pp


@contextlib.contextmanager
def p2g_config(pp, n_modes: int, path: int, block: int = 256, schedule: int = 0, per_cu: int = 0,
               brick: int = 4):
    """Select a P2G configuration for the block, then restore the default."""
    pp.polypic_set_p2g_config(n_modes, path, block, schedule, per_cu, brick)
    try:
        yield
    finally:
        pp.polypic_set_p2g_config(n_modes, -1, 256)


def note(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t) -> np.ndarray:
    return t.detach().cpu().numpy()


def rel(a, ref) -> float:
    return O.normwise_rel_err(a, ref)


def oracle_grid(pp_grid) -> O.Grid:
    return O.Grid(int(pp_grid.nx), int(pp_grid.ny), int(pp_grid.nz), float(pp_grid.dx),
                  float(pp_grid.inv_dx), tuple(float(v) for v in pp_grid.origin))


def ulp_ok(a, ref, n_ulp: float, scale: float) -> bool:
    """|a - ref| <= n_ulp float32 ulps of `scale` (the domain extent)."""
    return bool(np.all(np.abs(a.astype(np.float64) - ref.astype(np.float64))
                       <= n_ulp * np.spacing(np.float32(scale))))


def sample_nodes(gm: np.ndarray, k: int, seed: int) -> np.ndarray:
    """k flat node indices: half among occupied nodes, half anywhere."""
    rng = np.random.default_rng(seed)
    occ = np.flatnonzero(gm.ravel() > 0)
    pick = [rng.choice(occ, size=min(k // 2, occ.size), replace=False)] if occ.size else []
    pick.append(rng.integers(0, gm.size, size=k - (len(pick[0]) if pick else 0)))
    return np.unique(np.concatenate(pick))


def particles_touching(g: O.Grid, x: np.ndarray, nodes_flat: np.ndarray) -> np.ndarray:
    """Indices of the particles whose 3x3x3 stencil contains any of the given nodes.

    A node n is in the stencil of base node b iff n - 2 <= b <= n per axis, so the
    candidate base nodes of the sample are enumerated and matched in one pass.
    """
    b, _ = O.stencil_base(g, x)
    iz, rem = np.divmod(np.asarray(nodes_flat, np.int64), g.nx * g.ny)
    iy, ix = np.divmod(rem, g.nx)
    cand = []
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                bx, by, bz = ix - dx, iy - dy, iz - dz
                ok = (bx >= 0) & (by >= 0) & (bz >= 0)
                cand.append((bz[ok] * g.ny + by[ok]) * g.nx + bx[ok])
    cand = np.unique(np.concatenate(cand))
    flat_b = (b[2].astype(np.int64) * g.ny + b[1]) * g.nx + b[0]
    return np.flatnonzero(np.isin(flat_b, cand))
