"""FP64 oracle of the PolyPIC transfers on a staggered (MAC) grid -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import this module; the library never routes through it and shares no code with it.

The paper applies its transfers on marker-and-cell grids (section 3): each velocity
component alpha lives on its own faces, with the face mass m_{i alpha}, momentum
(mv)_{i alpha} and velocity v_{i alpha} of Table 1, and Eq. 1-8 and Eq. 13 are stated
per face.  Face alpha of node i sits at

    x_{i alpha} = origin + (i + (1 - e_alpha) / 2) dx,

i.e. on the node lattice along axis alpha and half a spacing up along the two other
axes (the usual staggering: x-velocities on the x-faces of the cells, and so on).
Each component is therefore a scalar transfer on its own shifted lattice, with its
own quadratic B-spline stencil, its own offsets t and therefore its own weights,
modes (Eq. 11, 14) and G2P projection (section 3.3):

* P2G (Eq. 1, 4, 13 per face): m_{i alpha} = sum_p m_p W_{ip alpha};
  (mv)_{i alpha} = sum_p m_p W_{ip alpha} sum_r c_{p r alpha} s_r(z_{i alpha}),
  z_{i alpha} = (x_{i alpha} - x_p) / dx at the particle's current position;
* grid update (Eq. 5 per face plus gravity and separating slip walls, as on the
  collocated grid; a face's wall test uses its index along its own axis, where faces
  and nodes coincide);
* G2P (Eq. 6-8 per face generalised as in section 3.3): c'_{p r alpha} =
  <v_alpha, s_r>_{W_alpha} / <s_r, s_r>_{W_alpha} over the face stencil of
  component alpha, K(t) cancelled on quadratic axes as in the collocated oracle;
* advection x' = x + dt c'_{p 0} and F' = (I + dt C) F with C_ab = c'_{a, 1+b} / dx.

The float32 stencil: u = fl32(fl32(x - o) * inv_dx) per axis; on an axis where
component alpha is staggered u' = fl32(u - 1/2) (exact for u < 2^22), else u' = u;
b = floor(fl32(u' - 1/2)) and t = u' - b - 1 in float64.  Arrays: face_mass,
face_mom and face_vel are (3, nz, ny, nx), component alpha's faces indexed like
the nodes (x fastest).

Parity pins: tests/test_oracle_mac.py.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

from .polypic_oracle import (ALLOWED_N_MODES, MODES, STENCIL, Grid, OracleRangeError,
                             clamp_bounds, phi_1d, projection_weights_1d, weights_1d)


def face_offset(alpha: int):
    """Position of face alpha relative to its node, in units of dx, per axis."""
    return tuple(0.0 if a == alpha else 0.5 for a in range(3))


def face_stencil(grid: Grid, x, alpha: int):
    """Base face b (int64, (3, P)) and offset t in [-1/2, 1/2) of component alpha."""
    x32 = np.asarray(x, np.float32)
    o32 = np.asarray(grid.origin, np.float32).reshape(3, 1)
    u = (x32 - o32) * np.float32(grid.inv_dx)          # two float32 roundings
    b = np.empty(u.shape, np.int64)
    t = np.empty(u.shape, np.float64)
    for a in range(3):
        ua = u[a] if a == alpha else u[a] - np.float32(0.5)   # exact subtraction
        ba = np.floor(ua - np.float32(0.5)).astype(np.int64)
        b[a] = ba
        t[a] = ua.astype(np.float64) - ba.astype(np.float64) - 1.0
    return b, t


def faces_in_range(grid: Grid, x) -> np.ndarray:
    """True where the stencils of all three components lie inside the face arrays."""
    ok = np.ones(np.asarray(x).shape[1], bool)
    for alpha in range(3):
        b, _ = face_stencil(grid, x, alpha)
        for a, n in enumerate(grid.dims):
            ok &= (b[a] >= 0) & (b[a] <= n - 3)
    return ok


def p2g(grid: Grid, x, coeff, n_modes: int, mass=None, uniform_mass: float = 1.0):
    """Face mass and momentum per component: returns (face_mass, face_mom), each
    (3, nz, ny, nx) float64 (entry alpha belongs to the faces of component alpha)."""
    if n_modes not in ALLOWED_N_MODES:
        raise ValueError("n_modes must be one of 1, 4, 8, 27")
    x = np.asarray(x)
    P = x.shape[1]
    if not np.all(faces_in_range(grid, x)):
        raise OracleRangeError("particle face stencil outside the grid")
    m = (np.full(P, float(uniform_mass)) if mass is None
         else np.asarray(mass).astype(np.float64))
    c = np.asarray(coeff)[:, :n_modes, :].astype(np.float64)
    nn = grid.n_nodes
    M = np.zeros((3, nn))
    Q = np.zeros((3, nn))
    for alpha in range(3):
        b, t = face_stencil(grid, x, alpha)
        w = [weights_1d(t[a]) for a in range(3)]
        ph = [phi_1d(t[a]) for a in range(3)]
        for jx, jy, jz in STENCIL:
            face = grid.flat(b[0] + jx, b[1] + jy, b[2] + jz)
            mW = m * w[0][jx] * w[1][jy] * w[2][jz]                 # m_{ip alpha}, Eq. 1
            V = np.zeros(P)
            for r in range(n_modes):
                kx, ky, kz = MODES[r]
                V += c[alpha, r] * (ph[0][kx][jx] * ph[1][ky][jy] * ph[2][kz][jz])
            M[alpha] += np.bincount(face, weights=mW, minlength=nn)
            Q[alpha] += np.bincount(face, weights=mW * V, minlength=nn)
    shape = (3, grid.nz, grid.ny, grid.nx)
    return M.reshape(shape), Q.reshape(shape)


def grid_update(grid: Grid, face_mass, face_mom, dt: float,
                gravity: Sequence[float] = (0.0, -9.8, 0.0), bc_layers: int = 1):
    """v_{i alpha} = (mv)_{i alpha} / m_{i alpha} + dt g_alpha where m_{i alpha} > 0, else 0;
    then, with bc_layers >= 1, v_alpha = 0 where it points into a wall: faces with index
    i_alpha <= 1 + bc_layers and v_alpha < 0, or i_alpha >= N_alpha - 1 - bc_layers and
    v_alpha > 0."""
    M = np.asarray(face_mass, np.float64)
    Q = np.asarray(face_mom, np.float64)
    v = np.zeros_like(Q)
    nz, ny, nx = M.shape[1:]
    idx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    along = (idx[2], idx[1], idx[0])
    for a in range(3):
        occ = M[a] > 0.0
        va = np.zeros(M.shape[1:])
        va[occ] = Q[a][occ] / M[a][occ] + dt * float(gravity[a])
        if bc_layers > 0:
            n = (nx, ny, nz)[a]
            lo = along[a] <= 1 + bc_layers
            hi = along[a] >= n - 1 - bc_layers
            va[lo & (va < 0.0)] = 0.0
            va[hi & (va > 0.0)] = 0.0
        v[a] = va
    return v


def g2p(grid: Grid, face_vel, x, n_modes: int, dt: float = 0.0, F=None):
    """c'_{p r alpha} = <v_alpha, s_r>_{W alpha} / <s_r, s_r>_{W alpha} for r < n_modes,
    each component over its own face stencil; then advection and the F update as on the
    collocated grid.  Returns (coeff_out (3, n_modes, P), x_out (3, P) float32, F_out)."""
    if n_modes not in ALLOWED_N_MODES:
        raise ValueError("n_modes must be one of 1, 4, 8, 27")
    x = np.asarray(x, np.float32)
    P = x.shape[1]
    if not np.all(faces_in_range(grid, x)):
        raise OracleRangeError("particle face stencil outside the grid")
    V = np.asarray(face_vel, np.float64).reshape(3, -1)
    c_out = np.zeros((3, n_modes, P))
    for alpha in range(3):
        b, t = face_stencil(grid, x, alpha)
        ph = [phi_1d(t[a]) for a in range(3)]
        q = [projection_weights_1d(t[a]) for a in range(3)]
        for r in range(n_modes):
            kx, ky, kz = MODES[r]
            num = np.zeros(P)
            den = np.zeros(P)
            for jx, jy, jz in STENCIL:
                face = grid.flat(b[0] + jx, b[1] + jy, b[2] + jz)
                qq = q[0][kx][jx] * q[1][ky][jy] * q[2][kz][jz]
                s = ph[0][kx][jx] * ph[1][ky][jy] * ph[2][kz][jz]
                num += qq * V[alpha, face]
                den += qq * s
            c_out[alpha, r] = num / den
    lo, hi = clamp_bounds(grid)
    x_new = (x.astype(np.float64) + dt * c_out[:, 0, :]).astype(np.float32)
    x_out = np.clip(x_new, lo.reshape(3, 1), hi.reshape(3, 1)).astype(np.float32)
    F_out = None
    if F is not None:
        F64 = np.asarray(F).astype(np.float64).reshape(3, 3, P)
        C = np.zeros((3, 3, P))
        if n_modes >= 4:
            for a in range(3):
                for bb in range(3):
                    C[a, bb] = c_out[a, 1 + bb] / grid.dx
        F_out = (F64 + dt * np.einsum("abp,bcp->acp", C, F64)).reshape(9, P)
    return c_out, x_out, F_out


def step(grid: Grid, x, coeff, n_modes: int, dt: float, gravity=(0.0, -9.8, 0.0),
         bc_layers: int = 1, mass=None, uniform_mass: float = 1.0, F=None, perm=None):
    """P2G -> grid update -> G2P on the faces.  With ``perm`` the G2P outputs are in that
    order (output i belongs to input particle perm[i]), as the library writes them."""
    x = np.asarray(x, np.float32)
    P = x.shape[1]
    perm = np.arange(P) if perm is None else np.asarray(perm)
    M, Q = p2g(grid, x, coeff, n_modes, mass, uniform_mass)
    v = grid_update(grid, M, Q, dt, gravity, bc_layers)
    Fs = None if F is None else np.asarray(F)[:, perm]
    c_out, x_out, F_out = g2p(grid, v, x[:, perm], n_modes, dt, Fs)
    return dict(face_mass=M, face_mom=Q, face_vel=v, coeff=c_out, x=x_out, F=F_out)
