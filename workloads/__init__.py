"""Seeded synthetic inputs for the PolyPIC transfer workloads.

This module only draws inputs: particle positions, masses, polynomial
coefficients, deformation gradients and grid geometry.  It holds none of the
transfer arithmetic, so both the FP64 oracle (under ``oracle/``) and the HIP
library can be fed from it without sharing any computation.

Conventions (the same for every workload):

* A grid of ``n`` cells per axis has spacing ``dx = 1/n``, origin 0 and
  ``n + 4`` nodes per axis: node ``i`` sits at ``i * dx`` and the domain is
  ``[2 dx, (n + 2) dx)`` (two guard nodes on each side, room for the 3-node
  quadratic B-spline stencil).  "Domain cell" ``c`` spans ``[(2 + c) dx,
  (3 + c) dx)``.
* Positions are SoA ``x[3][P]`` float32, coefficients ``coeff[3][27][P]``
  float32 in normalised units (mode ``r`` carries the factor
  ``dx**deg(r)``), deformation gradients ``F[9][P]`` row-major per particle.
* Random numbers come from ``numpy.random.default_rng(seed)`` (PCG64), drawn in
  the order positions -> velocities -> higher coefficients -> extras.  Small
  arrays are drawn in float64 and rounded to float32; the large coefficient
  planes are drawn directly in float32 (same distribution, less host memory).
* "Jittered" placement: each cell is split into ``sub`` sub-cells and one
  particle is placed uniformly at random inside each sub-cell.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

N_MODES_MAX = 27
GRAVITY = (0.0, -9.8, 0.0)  # y is up


@dataclasses.dataclass(frozen=True)
class GridSpec:
    """Collocated grid of ``cells`` domain cells per axis plus 2 guard nodes a side."""

    cells: Tuple[int, int, int]
    dx: float
    origin: Tuple[float, float, float] = (0.0, 0.0, 0.0)

    @property
    def nodes(self) -> Tuple[int, int, int]:
        """Node counts (nx, ny, nz) = cells + 4."""
        return tuple(c + 4 for c in self.cells)

    @property
    def inv_dx(self) -> float:
        return 1.0 / self.dx

    @property
    def n_nodes(self) -> int:
        nx, ny, nz = self.nodes
        return nx * ny * nz


def cubic_grid(n: int) -> GridSpec:
    return GridSpec(cells=(n, n, n), dx=1.0 / n)


@dataclasses.dataclass
class Scene:
    """One particle set on one grid, plus the step parameters of its workload."""

    name: str
    grid: GridSpec
    x: np.ndarray                 # (3, P) float32
    coeff: np.ndarray             # (3, 27, P) float32
    mass: Optional[np.ndarray]    # (P,) float32, or None for uniform mass
    uniform_mass: float = 1.0
    F: Optional[np.ndarray] = None  # (9, P) float32
    dt: float = 1e-4
    gravity: Tuple[float, float, float] = GRAVITY
    bc_layers: int = 1
    n_steps: int = 1

    @property
    def P(self) -> int:
        return int(self.x.shape[1])


def jittered_block(rng: np.random.Generator, grid: GridSpec, lo_cell, shape_cells,
                   sub=(2, 2, 2)) -> np.ndarray:
    """Positions (3, P) float32 of a block of domain cells, one particle per sub-cell.

    Cells are enumerated z-major, then y, then x; inside a cell the sub-cells in
    the same nesting.  P = prod(shape_cells) * prod(sub).
    """
    sh = [int(v) for v in shape_cells]
    sb = [int(v) for v in sub]
    P = int(np.prod(sh)) * int(np.prod(sb))
    jitter = rng.random((3, P))
    # index grid of shape (cz, cy, cx, sz, sy, sx), flattened in C order
    full = (sh[2], sh[1], sh[0], sb[2], sb[1], sb[0])
    x = np.empty((3, P), np.float32)
    for a in range(3):
        cell_axis = 2 - a          # position of this axis' cell index in `full`
        sub_axis = 5 - a           # position of this axis' sub-cell index
        shape = [1] * 6
        shape[cell_axis] = full[cell_axis]
        cidx = np.arange(full[cell_axis]).reshape(shape)
        shape = [1] * 6
        shape[sub_axis] = full[sub_axis]
        sidx = np.arange(full[sub_axis]).reshape(shape)
        fine = np.broadcast_to(cidx * sb[a] + sidx, full).reshape(-1)
        cell_coord = lo_cell[a] + (fine + jitter[a]) / sb[a]      # in domain cells
        x[a] = (grid.origin[a] + (2.0 + cell_coord) * grid.dx).astype(np.float32)
    return x


def _coefficients(rng: np.random.Generator, P: int, v_std: float, c_std: float,
                  zero: bool = False) -> np.ndarray:
    """coeff (3, 27, P): mode 0 (velocity) ~ N(0, v_std), modes 1..26 ~ N(0, c_std)."""
    c = np.zeros((3, N_MODES_MAX, P), np.float32)
    if zero:
        return c
    c[:, 0, :] = (rng.standard_normal((3, P)) * v_std).astype(np.float32)
    for a in range(3):
        hi = rng.standard_normal((N_MODES_MAX - 1, P), dtype=np.float32)
        hi *= np.float32(c_std)
        c[a, 1:, :] = hi
    return c


def config0(seed: int = 0) -> Scene:
    """Single-step parity case: 32^3 cells, 16^3-cell block at the centre, 8 ppc (32,768)."""
    rng = np.random.default_rng(seed)
    g = cubic_grid(32)
    x = jittered_block(rng, g, (8, 8, 8), (16, 16, 16), (2, 2, 2))
    c = _coefficients(rng, x.shape[1], 1.0, 0.1)
    return Scene("config0_32cube_32768", g, x, c, None, 1.0, dt=1e-4, bc_layers=0)


def config1(seed: int = 0, n: int = 128) -> Scene:
    """Dam break: 128^3 cells, block 64x128x64 cells at 8 ppc (4,194,304), at rest."""
    rng = np.random.default_rng(seed)
    g = cubic_grid(n)
    shape = (n // 2, n, n // 2)
    x = jittered_block(rng, g, (0, 0, 0), shape, (2, 2, 2))
    c = _coefficients(rng, x.shape[1], 1.0, 0.1, zero=True)
    return Scene(f"dambreak_{n}cube_{x.shape[1]}", g, x, c, None, 1.0, dt=1e-4,
                 bc_layers=1, n_steps=100)


def config1_moving(seed: int = 0, n: int = 128) -> Scene:
    """Dam-break geometry with non-trivial state: c0 ~ N(0,1), higher modes ~ N(0,0.1)."""
    s = config1(seed, n)
    rng = np.random.default_rng(seed + 1000)
    s.coeff = _coefficients(rng, s.P, 1.0, 0.1)
    s.name = s.name.replace("dambreak", "dambreak_moving")
    return s


def config2_fluid(seed: int = 0, n: int = 256, coefficients: bool = True) -> Scene:
    """Falling liquid block: 128x64x128 cells at 16 ppc (2x2x4 jitter) on a 256^3 grid.

    With coefficients=False the coefficient array is left empty (shape (3, 27, 0)) for
    callers that draw it elsewhere; the positions are the same either way."""
    rng = np.random.default_rng(seed)
    g = cubic_grid(n)
    q = n // 4
    x = jittered_block(rng, g, (q, n // 2, q), (n // 2, n // 4, n // 2), (2, 2, 4))
    c = (_coefficients(rng, x.shape[1], 1.0, 0.1) if coefficients
         else np.zeros((3, N_MODES_MAX, 0), np.float32))
    return Scene(f"fluid_{n}cube_{x.shape[1]}", g, x, c, None, 1.0, dt=1e-4, bc_layers=1)


def paper_dambreak_small(seed: int = 0, n: int = 64) -> Scene:
    """A dam break at the size of the paper's smallest fluid-only scene (section 4,
    Table 2: about 311 thousand particles, 8 modes, dt = 2e-4): a 36x36x30-cell block at
    8 ppc (311,040 particles) at the low corner of a 64^3-cell grid, at rest.  The
    paper's own scene geometry is not given; only its particle count, mode count and
    time step are matched."""
    rng = np.random.default_rng(seed)
    g = cubic_grid(n)
    x = jittered_block(rng, g, (0, 0, 0), (36, 36, 30), (2, 2, 2))
    c = _coefficients(rng, x.shape[1], 1.0, 0.1, zero=True)
    return Scene(f"paper_dambreak_{n}cube_{x.shape[1]}", g, x, c, None, 1.0, dt=2e-4,
                 bc_layers=1, n_steps=100)


def paper_dambreak_small_moving(seed: int = 0, n: int = 64) -> Scene:
    """The paper-size dam break with non-trivial state: c0 ~ N(0,1), higher modes ~ N(0,0.1)."""
    s = paper_dambreak_small(seed, n)
    rng = np.random.default_rng(seed + 1000)
    s.coeff = _coefficients(rng, s.P, 1.0, 0.1)
    s.name = s.name.replace("paper_dambreak", "paper_dambreak_moving")
    return s


def config2_fabric(seed: int = 0, n: int = 256, side: int = 1000) -> Scene:
    """Fabric sheet: side x side lattice, spacing dx/4, in the x-z plane at y = n/4 + 0.3 cells
    (64.3 cells on the 256^3 grid).

    Per-point mass = m_s + m_f with m_s = 1 and absorbed fluid m_f ~ U[0, 0.5];
    F = I + N(0, 0.01) per entry.
    """
    rng = np.random.default_rng(seed)
    g = cubic_grid(n)
    spacing = 0.25  # in cells
    extent = (side - 1) * spacing
    start = n / 2.0 - extent / 2.0
    ii, kk = np.meshgrid(np.arange(side), np.arange(side), indexing="ij")
    P = side * side
    x = np.empty((3, P), np.float32)
    x[0] = (g.origin[0] + (2.0 + start + kk.ravel() * spacing) * g.dx).astype(np.float32)
    x[1] = np.float32(g.origin[1] + (2.0 + n / 4.0 + 0.3) * g.dx)
    x[2] = (g.origin[2] + (2.0 + start + ii.ravel() * spacing) * g.dx).astype(np.float32)
    c = _coefficients(rng, P, 1.0, 0.1)
    m_f = rng.random(P) * 0.5
    mass = (1.0 + m_f).astype(np.float32)
    F = np.zeros((9, P), np.float32)
    F[:] = (rng.standard_normal((9, P)) * 0.01).astype(np.float32)
    F[0] += 1.0
    F[4] += 1.0
    F[8] += 1.0
    return Scene(f"fabric_{n}cube_{P}", g, x, c, mass, 1.0, F=F, dt=1e-4, bc_layers=1)


@dataclasses.dataclass
class MixtureScene:
    """Fluid particles and fabric points in one array on one grid (phase 0 / 1)."""

    name: str
    grid: GridSpec
    x: np.ndarray        # (3, P) float32
    coeff: np.ndarray    # (3, 27, P) float32
    phase: np.ndarray    # (P,) int32: 0 fluid, 1 solid
    mass_f: np.ndarray   # (P,) float32: fluid mass, or a fabric point's absorbed fluid
    mass_s: np.ndarray   # (P,) float32: solid mass (0 for fluid particles)
    F: np.ndarray        # (9, P) float32 (identity for fluid particles)
    dt: float = 1e-4
    gravity: Tuple[float, float, float] = GRAVITY
    bc_layers: int = 1

    @property
    def P(self) -> int:
        return int(self.x.shape[1])


def liquid_fabric_shared(seed: int = 0, n: int = 256, side: int = 1000) -> MixtureScene:
    """The liquid + fabric workload with both sets on ONE grid: the falling fluid block of
    config2_fluid (fluid mass 1) above the fabric sheet of config2_fabric (solid mass
    m_s = 1, absorbed fluid m_f ~ U[0, 0.5], F = I + N(0, 0.01)), fluid first.  Smaller n
    and side give the same layout at test sizes."""
    fl = config2_fluid(seed, n)
    fb = config2_fabric(seed, n, side)
    Pf, Pb = fl.P, fb.P
    x = np.concatenate([fl.x, fb.x], axis=1)
    c = np.concatenate([fl.coeff, fb.coeff], axis=2)
    phase = np.concatenate([np.zeros(Pf, np.int32), np.ones(Pb, np.int32)])
    mass_f = np.concatenate([np.ones(Pf, np.float32), (fb.mass - 1.0).astype(np.float32)])
    mass_s = np.concatenate([np.zeros(Pf, np.float32), np.ones(Pb, np.float32)])
    F = np.concatenate([np.tile(np.eye(3, dtype=np.float32).reshape(9, 1), (1, Pf)), fb.F],
                       axis=1)
    return MixtureScene(f"liquid_fabric_shared_{n}cube_{Pf}_{Pb}", fl.grid, x, c, phase,
                        mass_f, mass_s, F, dt=1e-4, bc_layers=1)


def config3_fd(seed: int = 0) -> Scene:
    """Small differentiable case: 16^3 cells, 8^3-cell central block, 8 ppc (4,096)."""
    rng = np.random.default_rng(seed)
    g = cubic_grid(16)
    x = jittered_block(rng, g, (4, 4, 4), (8, 8, 8), (2, 2, 2))
    c = _coefficients(rng, x.shape[1], 1.0, 0.1)
    return Scene("adjoint_16cube_4096", g, x, c, None, 1.0, dt=1e-4, bc_layers=1, n_steps=10)


def target_field_params(seed: int = 0, n_terms: int = 4):
    """Parameters of the seeded target velocity field v*(x) = sum_k A_k sin(2 pi kappa_k.x + phi_k).

    Returns (A (n_terms, 3), kappa (n_terms, 3) integer in 1..3, phi (n_terms,)).
    """
    rng = np.random.default_rng(10_000 + seed)
    A = rng.standard_normal((n_terms, 3))
    kappa = rng.integers(1, 4, size=(n_terms, 3)).astype(np.float64)
    phi = rng.random(n_terms) * 2.0 * math.pi
    return A, kappa, phi


def random_scene(seed: int, n: int, P: int, n_lo: int = 2, ppc_hint: int = 8,
                 v_std: float = 1.0, c_std: float = 0.1, mass_random: bool = False) -> Scene:
    """Uniformly scattered particles inside domain cells [n_lo, n - n_lo) per axis."""
    rng = np.random.default_rng(seed)
    g = cubic_grid(n)
    lo = g.origin[0] + (2.0 + n_lo) * g.dx
    hi = g.origin[0] + (2.0 + n - n_lo) * g.dx
    x = (lo + rng.random((3, P)) * (hi - lo)).astype(np.float32)
    c = _coefficients(rng, P, v_std, c_std)
    mass = (0.5 + rng.random(P)).astype(np.float32) if mass_random else None
    return Scene(f"random_{n}cube_{P}", g, x, c, mass, 1.0, dt=1e-4, bc_layers=1)


def batched_scenes(seed: int = 0, n_scenes: int = 64,
                   sizes=(64, 96, 128), p_lo: float = 1e4, p_hi: float = 2e6,
                   coefficients: bool = True) -> List[Scene]:
    """Many independent scenes with log-uniform particle counts at 8 ppc in random blocks.

    For each scene: n from ``sizes``; target particle count log-uniform in
    [p_lo, p_hi]; a block of about count/8 cells with aspect ratios in [1/2, 2],
    placed uniformly at random inside the domain (n is redrawn if it does not fit).
    The realised count is 8 * (block volume).  With coefficients=False the
    coefficient arrays are left empty (shape (3, 27, 0)) for callers that draw
    them elsewhere; positions are the same either way.
    """
    rng = np.random.default_rng(seed)
    crng = np.random.default_rng(20_000 + seed)   # coefficients: a stream of their own
    scenes = []
    for s in range(n_scenes):
        target = math.exp(rng.uniform(math.log(p_lo), math.log(p_hi)))
        cells = max(1.0, target / 8.0)
        ra, rb = rng.uniform(0.5, 2.0, size=2)
        while True:
            n = int(rng.choice(sizes))
            base = (cells / (ra * rb)) ** (1.0 / 3.0)
            dims = [max(1, int(round(base * ra))), max(1, int(round(base * rb))),
                    max(1, int(round(base)))]
            if all(d <= n for d in dims):
                break
            ra, rb = rng.uniform(0.5, 2.0, size=2)
        g = cubic_grid(n)
        lo = [int(rng.integers(0, n - d + 1)) for d in dims]
        x = jittered_block(rng, g, lo, dims, (2, 2, 2))
        c = (_coefficients(crng, x.shape[1], 1.0, 0.1) if coefficients
             else np.zeros((3, N_MODES_MAX, 0), np.float32))
        scenes.append(Scene(f"batch{s}_{n}cube_{x.shape[1]}", g, x, c, None, 1.0,
                            dt=1e-4, bc_layers=1, n_steps=10))
    return scenes
