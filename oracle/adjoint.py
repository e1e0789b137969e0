"""FP64 differentiable twin of the transfer step -- TEST INFRASTRUCTURE ONLY.

Reference for the hand-written adjoint of the HIP library.  The step of
``polypic_oracle`` (P2G of Eq. 1, 4, 13; grid update of Eq. 5 with gravity and
slip walls; G2P as the weighted least-squares fit of section 3.3; advection)
is restated with plain torch CPU float64 operations so that torch.autograd
gives its exact gradient.  Differences from ``polypic_oracle.step``, all on
purpose:

* positions stay float64 (the library rounds them to float32; rounding has
  derivative 1 almost everywhere);
* the stencil base b = floor(u - 1/2) is computed in float64 and treated as a
  constant (it is piecewise constant in x);
* no sort: results are in input order.

The forward values are pinned against ``polypic_oracle`` and the gradients
against central finite differences in the tests.  Quantities follow the
paper's notation where it has one (m_p, c_pra, w_ip, s_r).
"""
from __future__ import annotations

import itertools
import math
from typing import Sequence, Tuple

import torch

from .polypic_oracle import MODES, Grid

STENCIL = tuple(itertools.product(range(3), repeat=3))  # (jx, jy, jz)


def _factors(t: torch.Tensor):
    """Per-axis 1-D factors at nodes j = 0, 1, 2: weights w, zhat, ghat (Eq. 14 reading)."""
    z = [j - 1.0 - t for j in range(3)]
    # quadratic B-spline at the node offsets (|zhat_0|, |zhat_2| in [1/2, 3/2), |zhat_1| <= 1/2)
    w = [0.5 * (1.5 - (1.0 + t)) ** 2, 0.75 - t * t, 0.5 * (1.5 - (1.0 - t)) ** 2]
    a = t * (1.0 - 4.0 * t * t)
    g = [zj * zj - a * zj - 0.25 for zj in z]
    return w, z, g


def _stencil(grid: Grid, x: torch.Tensor):
    """Base node (int64, detached) and t = u - b - 1 (differentiable) per axis."""
    o = torch.tensor(grid.origin, dtype=torch.float64).reshape(3, 1)
    u = (x - o) * grid.inv_dx
    b = torch.floor(u.detach() - 0.5).to(torch.int64)
    t = u - b.to(torch.float64) - 1.0
    return b, t


def _flat(grid: Grid, b, j):
    return ((b[2] + j[2]) * grid.ny + (b[1] + j[1])) * grid.nx + (b[0] + j[0])


def _mode_index(n_modes: int):
    """Per-axis indices (kx_r, ky_r, kz_r) of the first n_modes modes."""
    return (torch.tensor([MODES[r][0] for r in range(n_modes)]),
            torch.tensor([MODES[r][1] for r in range(n_modes)]),
            torch.tensor([MODES[r][2] for r in range(n_modes)]))


def _tables(t: torch.Tensor):
    """Per-axis tables over (factor k, node j, particle p): the weights w_j, the mode
    factors phi_k(j) = 1, zhat, ghat (Eq. 11, 14) and the G2P projection rows
    w, w zhat, (1, -2, 1) (K(t) cancelled on quadratic axes)."""
    wt, phit, qt = [], [], []
    for a in range(3):
        w, z, g = (torch.stack(f) for f in _factors(t[a]))  # (3 j, P): w_j, zhat_j, ghat_j
        one = torch.ones_like(w)
        wt.append(w)
        phit.append(torch.stack([one, z, g]))
        qt.append(torch.stack([w, w * z, torch.stack([one[0], -2.0 * one[1], one[2]])]))
    return wt, phit, qt


def _mode_rows(f, j, n_modes: int):
    """(n_modes, P): f_x[kx_r, jx] f_y[ky_r, jy] f_z[kz_r, jz] at stencil node j."""
    KX, KY, KZ = _mode_index(n_modes)
    return f[0][KX, j[0]] * f[1][KY, j[1]] * f[2][KZ, j[2]]


def p2g(grid: Grid, x: torch.Tensor, c: torch.Tensor, n_modes: int,
        mass: torch.Tensor = None, uniform_mass: float = 1.0):
    """P2G (Eq. 1, 4, 13): m_i = sum_p m_p W_ip;  p_i = sum_p m_p W_ip sum_r c_pr s_r(i).

    Returns (M (n_nodes,), Q (3, n_nodes)), flat node index x fastest."""
    P = x.shape[1]
    m = mass if mass is not None else torch.full((P,), float(uniform_mass), dtype=torch.float64)
    b, t = _stencil(grid, x)
    wt, phit, _ = _tables(t)
    nn = grid.n_nodes
    M = torch.zeros(nn, dtype=torch.float64)
    Q = torch.zeros(3, nn, dtype=torch.float64)
    for j in STENCIL:
        node = _flat(grid, b, j)
        mW = m * wt[0][j[0]] * wt[1][j[1]] * wt[2][j[2]]    # m_p W_ip
        V = (c * _mode_rows(phit, j, n_modes)).sum(dim=1)   # sum_r c_par s_r(j): (3, P)
        M = M.index_add(0, node, mW)
        Q = Q.index_add(1, node, mW * V)
    return M, Q


def grid_update(grid: Grid, M: torch.Tensor, Q: torch.Tensor, dt: float,
                gravity: Sequence[float] = (0.0, -9.8, 0.0), bc_layers: int = 1,
                nodes: torch.Tensor = None):
    """Grid update (Eq. 5 + gravity + separating slip walls) of M (n,), Q (3, n).

    ``nodes`` gives the flat index of each entry when M and Q hold a subset of the
    grid's nodes (default: all nodes in order); it only places the walls."""
    occ = M > 0
    Msafe = torch.where(occ, M, torch.ones_like(M))
    gvec = torch.tensor(gravity, dtype=torch.float64).reshape(3, 1)
    v = torch.where(occ, Q / Msafe + dt * gvec, torch.zeros_like(Q))
    if bc_layers > 0:
        idx = torch.arange(grid.n_nodes) if nodes is None else torch.as_tensor(nodes)
        ix = idx % grid.nx
        iy = (idx // grid.nx) % grid.ny
        iz = idx // (grid.nx * grid.ny)
        along = (ix, iy, iz)
        rows = []
        for a, n in enumerate(grid.dims):
            va = v[a]
            lo = along[a] <= 1 + bc_layers
            hi = along[a] >= n - 1 - bc_layers
            va = torch.where(lo & (va < 0), torch.zeros_like(va), va)
            va = torch.where(hi & (va > 0), torch.zeros_like(va), va)
            rows.append(va)
        v = torch.stack(rows)
    return v


def g2p(grid: Grid, v: torch.Tensor, x: torch.Tensor, n_modes: int, dt: float):
    """G2P and advection: c'_r = <v, s_r>_W / <s_r, s_r>_W (K(t) cancelled on quadratic
    axes), x' = x + dt c'_0 kept inside [o + 2 dx, o + (N - 2) dx].  v is (3, n_nodes)."""
    P = x.shape[1]
    b, t = _stencil(grid, x)
    _, phit, qt = _tables(t)
    num = torch.zeros(3, n_modes, P, dtype=torch.float64)
    den = torch.zeros(n_modes, P, dtype=torch.float64)
    for j in STENCIL:
        qq = _mode_rows(qt, j, n_modes)                     # projection weight: (n_modes, P)
        num = num + qq * v[:, _flat(grid, b, j)].unsqueeze(1)
        den = den + qq * _mode_rows(phit, j, n_modes)
    c_out = num / den
    lo = torch.tensor([grid.origin[a] + 2 * grid.dx for a in range(3)],
                      dtype=torch.float64).reshape(3, 1)
    hi = torch.tensor([grid.origin[a] + (n - 2) * grid.dx for a, n in enumerate(grid.dims)],
                      dtype=torch.float64).reshape(3, 1)
    x_out = torch.minimum(torch.maximum(x + dt * c_out[:, 0, :], lo), hi)
    return x_out, c_out


def step(grid: Grid, x: torch.Tensor, c: torch.Tensor, n_modes: int, dt: float,
         gravity: Sequence[float] = (0.0, -9.8, 0.0), bc_layers: int = 1,
         mass: torch.Tensor = None, uniform_mass: float = 1.0):
    """One differentiable step: (x (3, P), c (3, n_modes, P)) -> (x', c', grid dict):
    P2G, grid update, G2P with advection, in that order."""
    M, Q = p2g(grid, x, c, n_modes, mass, uniform_mass)
    v = grid_update(grid, M, Q, dt, gravity, bc_layers)
    x_out, c_out = g2p(grid, v, x, n_modes, dt)
    return x_out, c_out, dict(grid_mass=M, grid_mom=Q, grid_vel=v)


def target_field(x: torch.Tensor, A, kappa, phase) -> torch.Tensor:
    """v*(x) = sum_k A_k sin(2 pi kappa_k . x + phi_k), (3, P)."""
    A = torch.as_tensor(A, dtype=torch.float64)
    kappa = torch.as_tensor(kappa, dtype=torch.float64)
    phase = torch.as_tensor(phase, dtype=torch.float64)
    arg = 2 * math.pi * (kappa @ x) + phase.reshape(-1, 1)  # (K, P)
    return A.T @ torch.sin(arg)


def loss(x: torch.Tensor, c: torch.Tensor, A, kappa, phase) -> torch.Tensor:
    """L = 1/2 sum_p || c_p0 - v*(x_p) ||^2 on the final particle state."""
    d = c[:, 0, :] - target_field(x, A, kappa, phase)
    return 0.5 * (d * d).sum()


def rollout(grid: Grid, x0, c0, n_modes: int, n_steps: int, dt: float, gravity, bc_layers,
            mass=None, uniform_mass: float = 1.0) -> Tuple[torch.Tensor, torch.Tensor]:
    x, c = x0, c0
    for _ in range(n_steps):
        x, c, _ = step(grid, x, c, n_modes, dt, gravity, bc_layers, mass, uniform_mass)
    return x, c


def loss_and_grad(grid: Grid, x0, c0, n_modes: int, n_steps: int, dt: float, gravity,
                  bc_layers, target, mass=None, uniform_mass: float = 1.0):
    """Loss after n_steps and its gradient w.r.t. x0 (3, P), c0 (3, n_modes, P) and mass."""
    x = torch.as_tensor(x0, dtype=torch.float64).clone().requires_grad_(True)
    c = torch.as_tensor(c0, dtype=torch.float64).clone().requires_grad_(True)
    m = None
    if mass is not None:
        m = torch.as_tensor(mass, dtype=torch.float64).clone().requires_grad_(True)
    xs, cs = rollout(grid, x, c, n_modes, n_steps, dt, gravity, bc_layers, m, uniform_mass)
    L = loss(xs, cs, *target)
    inputs = [x, c] + ([m] if m is not None else [])
    grads = torch.autograd.grad(L, inputs)
    return float(L.detach()), grads
