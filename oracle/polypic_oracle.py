"""FP64 CPU oracle of the PolyPIC transfers -- TEST INFRASTRUCTURE ONLY.

This module is the plain, slow reference that the HIP library is checked
against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import it; the library never routes through it.  It
shares no code with the HIP path.

What it computes (Dennison & Maddock, "Using The Polynomial Particle-in-Cell
Method for Liquid-Fabric Interaction", section 3), on a collocated grid:

* P2G, Eq. 1 and 4 (mass) and Eq. 13 (momentum carried by the polynomial
  modes), summed over particles as in Eq. 3;
* the grid velocity of Eq. 5 plus a light explicit update (gravity and
  separating slip walls -- not in the paper, which defers the grid solve to
  the model of Fei et al.);
* G2P, Eq. 6-8 generalised to the weighted least-squares fit of the modes
  that section 3.3 takes from Fu et al.  With the w-orthogonal basis of
  Eq. 11 and Eq. 14 the fit decouples into one ratio per mode;
* advection x' = x + dt v_p and, for material points, F' = (I + dt C) F.

Readings of the paper that this file fixes (each is also listed in the
design notes of the repository):

* N(x) is the quadratic B-spline (section 3.1 leaves the kernel unnamed).
* Modes are evaluated at zhat = (x_i - x_p)/dx at the particle's current
  position (identity map in place of the affine map of Eq. 12) and the
  coefficients are stored in these normalised units.
* Eq. 14 is read as g(z) = z^2 - a z - dx^2/4 with a = delta (dx^2 - 4 delta^2)
  / dx^2, where z = x_i - x_p and delta = x_p - (nearest node).  In units of dx
  this is ghat(zhat) = zhat^2 - t (1 - 4 t^2) zhat - 1/4 with t = delta/dx.
* The modes are the tensor products phi_kx(zx) phi_ky(zy) phi_kz(zz) with
  phi_0 = 1, phi_1 = zhat, phi_2 = ghat, in the graded order MODES below, so
  that N_r = 1, 4, 8, 27 is PIC, APIC, multilinear, full.
* G2P coefficient of mode r is <v, s_r>_W / <s_r, s_r>_W with W = w_x w_y w_z.
  On an axis where the mode is quadratic, w_j ghat_j = K(t) (1, -2, 1)_j with
  K(t) = (1 - 4t^2)^2 (3 - 4t^2) / 32, so K cancels between numerator and
  denominator; the cancelled form is used for every t, which also defines the
  coefficient at the degenerate t = -1/2 (K = 0) by continuity.
* The stencil base is computed from float32 inputs by exactly specified
  float32 operations (u = (x - o) * inv_dx, b = floor(u - 1/2)); everything
  after that is float64.
"""
from __future__ import annotations

import dataclasses
import itertools
from typing import Optional, Sequence, Tuple

import numpy as np

# Graded mode order: index r -> (kx, ky, kz); phi_0 = 1, phi_1 = zhat, phi_2 = ghat.
MODES: Tuple[Tuple[int, int, int], ...] = (
    (0, 0, 0),
    (1, 0, 0), (0, 1, 0), (0, 0, 1),
    (1, 1, 0), (1, 0, 1), (0, 1, 1),
    (1, 1, 1),
    (2, 0, 0), (0, 2, 0), (0, 0, 2),
    (2, 1, 0), (2, 0, 1), (1, 2, 0), (0, 2, 1), (1, 0, 2), (0, 1, 2),
    (2, 1, 1), (1, 2, 1), (1, 1, 2),
    (2, 2, 0), (2, 0, 2), (0, 2, 2),
    (2, 2, 1), (2, 1, 2), (1, 2, 2),
    (2, 2, 2),
)
ALLOWED_N_MODES = (1, 4, 8, 27)
STENCIL = tuple(itertools.product(range(3), repeat=3))  # (jx, jy, jz)


class OracleRangeError(ValueError):
    """A particle's 3x3x3 stencil leaves the grid storage."""


@dataclasses.dataclass(frozen=True)
class Grid:
    """Collocated grid: node (ix, iy, iz) at origin + (ix, iy, iz) * dx."""

    nx: int
    ny: int
    nz: int
    dx: float
    inv_dx: float
    origin: Tuple[float, float, float] = (0.0, 0.0, 0.0)

    @property
    def dims(self) -> Tuple[int, int, int]:
        return (self.nx, self.ny, self.nz)

    @property
    def n_nodes(self) -> int:
        return self.nx * self.ny * self.nz

    def flat(self, ix, iy, iz):
        """Flat node index, x fastest."""
        return (np.asarray(iz, np.int64) * self.ny + iy) * self.nx + ix


def grid_from_spec(spec) -> Grid:
    """Grid from a ``workloads.GridSpec`` (duck-typed: nodes, dx, inv_dx, origin)."""
    nx, ny, nz = spec.nodes
    return Grid(nx, ny, nz, float(spec.dx), float(spec.inv_dx), tuple(spec.origin))


# ---------------------------------------------------------------- stencil (section 3.1)

def quadratic_bspline(d):
    """N(d): the quadratic B-spline, 3/4 - d^2 for |d| < 1/2, (3/2 - |d|)^2 / 2 for
    1/2 <= |d| < 3/2, else 0.  Section 3.1 uses an unnamed N(x); this is the reading."""
    a = np.abs(np.asarray(d, np.float64))
    return np.where(a < 0.5, 0.75 - a * a, np.where(a < 1.5, 0.5 * (1.5 - a) ** 2, 0.0))


def stencil_base(grid: Grid, x):
    """Base node b (int64, (3, P)) and offset t = u - b - 1 in [-1/2, 1/2) (float64).

    u = fl32(fl32(x - o) * inv_dx) per axis and b = floor(fl32(u - 1/2)), all in
    float32 with round-to-nearest; node b + 1 is the nearest node and the
    stencil is nodes b, b + 1, b + 2.
    """
    x32 = np.asarray(x, np.float32)
    o32 = np.asarray(grid.origin, np.float32).reshape(3, 1)
    u = (x32 - o32) * np.float32(grid.inv_dx)          # two float32 roundings
    b = np.floor(u - np.float32(0.5)).astype(np.int64)  # exact for u < 2^22
    t = u.astype(np.float64) - b.astype(np.float64) - 1.0
    return b, t


def stencil_in_range(grid: Grid, b) -> np.ndarray:
    """True where 0 <= b_axis <= N_axis - 3 on every axis."""
    ok = np.ones(b.shape[1], bool)
    for a, n in enumerate(grid.dims):
        ok &= (b[a] >= 0) & (b[a] <= n - 3)
    return ok


def node_offsets(t):
    """zhat_j = (x_i - x_p)/dx = j - 1 - t for the stencil nodes j = 0, 1, 2."""
    return [np.asarray(j - 1.0 - t, np.float64) for j in range(3)]


def weights_1d(t):
    """w_j = N(zhat_j) for j = 0, 1, 2 (section 3.1, w_ip = N(x_p - x_i))."""
    return [quadratic_bspline(z) for z in node_offsets(t)]


def ghat_1d(t):
    """Orthogonalised quadratic of Eq. 14 (reading above) at the 3 stencil nodes."""
    a = t * (1.0 - 4.0 * t * t)
    return [z * z - a * z - 0.25 for z in node_offsets(t)]


def phi_1d(t):
    """phi[k][j] for k = 0 (constant), 1 (zhat), 2 (ghat): the 1-D factors of Eq. 11."""
    z = node_offsets(t)
    g = ghat_1d(t)
    one = [np.ones_like(z[0]) for _ in range(3)]
    return [one, z, g]


def projection_weights_1d(t):
    """q[k][j]: the 1-D weight of the G2P inner product with K(t) cancelled on ghat.

    q_0 = w, q_1 = w zhat, q_2 = (1, -2, 1) = w ghat / K(t).
    """
    w = weights_1d(t)
    z = node_offsets(t)
    ones = np.ones_like(w[0])
    return [w, [w[j] * z[j] for j in range(3)], [ones, -2.0 * ones, ones]]


# ---------------------------------------------------------------- sort key (not in the paper)

def morton_key(b) -> np.ndarray:
    """Morton code of the base node: bit k of b_x, b_y, b_z -> key bits 3k, 3k+1, 3k+2."""
    b = np.asarray(b, np.int64)
    key = np.zeros(b.shape[1], np.uint64)
    for bit in range(11):
        for a in range(3):
            key |= (((b[a] >> bit) & 1).astype(np.uint64)) << np.uint64(3 * bit + a)
    return key.astype(np.uint32)


def sort_keys(grid: Grid, x):
    """Cell keys of every particle and the stable permutation that sorts them.

    Returns (keys_sorted uint32 (P,), perm int32 (P,)) with
    keys_sorted[i] = key[perm[i]]; ties keep input order.
    """
    b, _ = stencil_base(grid, x)
    if not np.all(stencil_in_range(grid, b)):
        raise OracleRangeError("particle stencil outside the grid")
    key = morton_key(b)
    perm = np.argsort(key, kind="stable")
    return key[perm], perm.astype(np.int32)


# ---------------------------------------------------------------- P2G (Eq. 1, 3, 4, 13)

def p2g(grid: Grid, x, coeff, n_modes: int, mass=None, uniform_mass: float = 1.0):
    """Grid mass m_i = sum_p m_p W_ip and momentum (mv)_ia = sum_p m_p W_ip sum_r c_par s_r.

    x: (3, P) float32; coeff: (3, >= n_modes, P); mass: (P,) or None.
    Returns (grid_mass (nz, ny, nx), grid_mom (3, nz, ny, nx)) in float64.
    """
    if n_modes not in ALLOWED_N_MODES:
        raise ValueError("n_modes must be one of 1, 4, 8, 27")
    x = np.asarray(x)
    P = x.shape[1]
    b, t = stencil_base(grid, x)
    if not np.all(stencil_in_range(grid, b)):
        raise OracleRangeError("particle stencil outside the grid")
    # inputs are used at the precision they come in (float32 from the library's
    # callers, float64 in the exact-reproduction pins)
    m = (np.full(P, float(uniform_mass)) if mass is None
         else np.asarray(mass).astype(np.float64))
    c = np.asarray(coeff)[:, :n_modes, :].astype(np.float64)
    w = [weights_1d(t[a]) for a in range(3)]
    ph = [phi_1d(t[a]) for a in range(3)]
    nn = grid.n_nodes
    M = np.zeros(nn)
    Q = np.zeros((3, nn))
    for jx, jy, jz in STENCIL:
        node = grid.flat(b[0] + jx, b[1] + jy, b[2] + jz)
        mW = m * w[0][jx] * w[1][jy] * w[2][jz]            # m_ip, Eq. 1
        V = np.zeros((3, P))
        for r in range(n_modes):
            kx, ky, kz = MODES[r]
            s = ph[0][kx][jx] * ph[1][ky][jy] * ph[2][kz][jz]  # s_r at node i, Eq. 11
            V += c[:, r, :] * s
        M += np.bincount(node, weights=mW, minlength=nn)
        for a in range(3):
            Q[a] += np.bincount(node, weights=mW * V[a], minlength=nn)
    shape = (grid.nz, grid.ny, grid.nx)
    return M.reshape(shape), Q.reshape((3,) + shape)


# ---------------------------------------------------------------- P2G with the affine map (Eq. 12-13)

def p2g_affine(grid: Grid, x, coeff, n_modes: int, dt: float, x_fit=None, mass=None,
               uniform_mass: float = 1.0):
    """P2G with the modes evaluated through the affine back-map of Eq. 12.

    The coefficients of a particle were fitted (G2P) at its previous position x_fit, in
    the basis orthogonalised there; the particle has since moved to x.  Eq. 12 maps the
    present configuration back to that one, xi(x) = x_fit + (I + dt C)^-1 (x - x_p), so
    the mode argument of Eq. 13 at node i is, in units of dx,

        z'_i = (I + dt C)^-1 (x_i - x_p) / dx,

    with C the particle's velocity-gradient matrix taken from its linear coefficients
    (C_ab = c_{a, 1+b} / dx; C = 0 below 4 modes), and the quadratic factor of Eq. 14 is
    the one of the fitting configuration: ghat(z) = z^2 - a z - 1/4 with
    a = t_fit (1 - 4 t_fit^2), t_fit the offset of x_fit from its nearest node.  Without
    x_fit the present offset is used.  The weights W_ip stay those of the present position
    (Eq. 1 and 13 use m_ip of the present configuration).

    Returns (grid_mass, grid_mom) like ``p2g``.
    """
    if n_modes not in ALLOWED_N_MODES:
        raise ValueError("n_modes must be one of 1, 4, 8, 27")
    x = np.asarray(x)
    P = x.shape[1]
    b, t = stencil_base(grid, x)
    if not np.all(stencil_in_range(grid, b)):
        raise OracleRangeError("particle stencil outside the grid")
    if x_fit is None:
        t_fit = t
    else:
        _, t_fit = stencil_base(grid, x_fit)
    a_fit = t_fit * (1.0 - 4.0 * t_fit * t_fit)           # Eq. 14 (reading), per axis
    m = (np.full(P, float(uniform_mass)) if mass is None
         else np.asarray(mass).astype(np.float64))
    c = np.asarray(coeff)[:, :n_modes, :].astype(np.float64)
    # A = I + dt C per particle and its inverse (Eq. 12)
    A = np.repeat(np.eye(3)[None], P, axis=0)
    if n_modes >= 4:
        for al in range(3):
            for be in range(3):
                A[:, al, be] += dt * c[al, 1 + be] / grid.dx
    Ainv = np.linalg.inv(A)
    w = [weights_1d(t[a]) for a in range(3)]
    zs = [node_offsets(t[a]) for a in range(3)]
    nn = grid.n_nodes
    M = np.zeros(nn)
    Q = np.zeros((3, nn))
    for jx, jy, jz in STENCIL:
        node = grid.flat(b[0] + jx, b[1] + jy, b[2] + jz)
        mW = m * w[0][jx] * w[1][jy] * w[2][jz]
        zhat = np.stack([zs[0][jx], zs[1][jy], zs[2][jz]])       # (3, P)
        zp = np.einsum("pab,bp->ap", Ainv, zhat)                  # z'_i, (3, P)
        phi = [[np.ones(P), zp[a], zp[a] * zp[a] - a_fit[a] * zp[a] - 0.25] for a in range(3)]
        V = np.zeros((3, P))
        for r in range(n_modes):
            kx, ky, kz = MODES[r]
            V += c[:, r, :] * (phi[0][kx] * phi[1][ky] * phi[2][kz])
        M += np.bincount(node, weights=mW, minlength=nn)
        for al in range(3):
            Q[al] += np.bincount(node, weights=mW * V[al], minlength=nn)
    shape = (grid.nz, grid.ny, grid.nx)
    return M.reshape(shape), Q.reshape((3,) + shape)


# ---------------------------------------------------------------- grid update (Eq. 5 + walls)

def grid_update(grid: Grid, grid_mass, grid_mom, dt: float,
                gravity: Sequence[float] = (0.0, -9.8, 0.0), bc_layers: int = 1):
    """v_i = (mv)_i / m_i + dt g where m_i > 0, else 0 (Eq. 5); then separating slip walls.

    Walls (bc_layers >= 1), per axis with storage index i along it: v_axis is set
    to 0 where i <= 1 + bc_layers and v_axis < 0, and where
    i >= N_axis - 1 - bc_layers and v_axis > 0.  bc_layers = 0: no walls.
    """
    M = np.asarray(grid_mass, np.float64)
    Q = np.asarray(grid_mom, np.float64)
    v = np.zeros_like(Q)
    occ = M > 0.0
    for a in range(3):
        va = np.zeros_like(M)
        va[occ] = Q[a][occ] / M[occ] + dt * float(gravity[a])
        v[a] = va
    if bc_layers > 0:
        nz, ny, nx = M.shape
        idx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        along = (idx[2], idx[1], idx[0])  # axis 0 = x -> last array index
        for a, n in enumerate((nx, ny, nz)):
            lo = along[a] <= 1 + bc_layers
            hi = along[a] >= n - 1 - bc_layers
            v[a][lo & (v[a] < 0.0)] = 0.0
            v[a][hi & (v[a] > 0.0)] = 0.0
    return v


# ---------------------------------------------------------------- G2P (Eq. 6-8, section 3.3)

def clamp_bounds(grid: Grid):
    """Per-axis float32 bounds [lo, hi] keeping positions in [o + 2 dx, o + (N - 2) dx)."""
    lo = np.empty(3, np.float32)
    hi = np.empty(3, np.float32)
    for a, n in enumerate(grid.dims):
        lo[a] = np.float32(grid.origin[a] + 2.0 * grid.dx)
        top = np.float32(grid.origin[a] + (n - 2) * grid.dx)
        hi[a] = np.nextafter(top, np.float32(-np.inf))
    return lo, hi


def g2p(grid: Grid, grid_vel, x, n_modes: int, dt: float = 0.0, F=None):
    """Coefficients c'_par = <v_a, s_r>_W / <s_r, s_r>_W for r < n_modes, then advection.

    grid_vel: (3, nz, ny, nx); x: (3, P) float32.
    Returns (coeff_out (3, n_modes, P) float64, x_out (3, P) float32,
    F_out (9, P) float64 or None).  x_out = clamp(fl32(x + dt c'_p0)).
    F_out = (I + dt C) F with C_ab = c'_{a, 1+b} / dx (needs n_modes >= 4).
    """
    if n_modes not in ALLOWED_N_MODES:
        raise ValueError("n_modes must be one of 1, 4, 8, 27")
    x = np.asarray(x, np.float32)
    P = x.shape[1]
    b, t = stencil_base(grid, x)
    if not np.all(stencil_in_range(grid, b)):
        raise OracleRangeError("particle stencil outside the grid")
    V = np.asarray(grid_vel, np.float64).reshape(3, -1)
    ph = [phi_1d(t[a]) for a in range(3)]
    q = [projection_weights_1d(t[a]) for a in range(3)]
    nodes = {}
    for j in STENCIL:
        nodes[j] = grid.flat(b[0] + j[0], b[1] + j[1], b[2] + j[2])
    c_out = np.zeros((3, n_modes, P))
    for r in range(n_modes):
        kx, ky, kz = MODES[r]
        num = np.zeros((3, P))
        den = np.zeros(P)
        for j in STENCIL:
            jx, jy, jz = j
            qq = q[0][kx][jx] * q[1][ky][jy] * q[2][kz][jz]
            s = ph[0][kx][jx] * ph[1][ky][jy] * ph[2][kz][jz]
            num += qq * V[:, nodes[j]]
            den += qq * s
        c_out[:, r, :] = num / den
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
        # F' = F + dt C F
        F_new = F64 + dt * np.einsum("abp,bcp->acp", C, F64)
        F_out = F_new.reshape(9, P)
    return c_out, x_out, F_out


# ---------------------------------------------------------------- shared-grid mixture (section 3.4)

FLUID, SOLID = 0, 1


def _phase_masses(phase, mass_f, mass_s):
    """Per-particle transfer mass: m_f for a fluid particle (Eq. 15), m_s + m_f for a solid
    particle with its absorbed fluid (Eq. 18)."""
    phase = np.asarray(phase)
    if np.any((phase != FLUID) & (phase != SOLID)):
        raise ValueError("phase must be 0 (fluid) or 1 (solid)")
    mf = np.asarray(mass_f).astype(np.float64)
    ms = np.zeros_like(mf) if mass_s is None else np.asarray(mass_s).astype(np.float64)
    return phase, np.where(phase == SOLID, ms + mf, mf)


def mixture_p2g(grid: Grid, x, coeff, n_modes: int, phase, mass_f, mass_s=None):
    """Liquid and fabric particles on one grid (section 3.4): each node carries a fluid
    set of channels (m_f, m_f v_f; Eq. 15-16, fluid particles only, mass m_f) and a solid
    set (mixture mass and momentum; Eq. 18-19, solid particles only, mass m_s + m_f with
    the absorbed fluid).  Returns (grid_mass (2, nz, ny, nx), grid_mom (2, 3, nz, ny, nx)),
    index 0 the fluid set and 1 the solid one."""
    phase, m = _phase_masses(phase, mass_f, mass_s)
    x = np.asarray(x)
    c = np.asarray(coeff)
    M = np.zeros((2, grid.nz, grid.ny, grid.nx))
    Q = np.zeros((2, 3, grid.nz, grid.ny, grid.nx))
    for k in (FLUID, SOLID):
        sel = np.flatnonzero(phase == k)
        M[k], Q[k] = p2g(grid, x[:, sel], c[:, :, sel], n_modes, m[sel])
    return M, Q


def mixture_grid_update(grid: Grid, grid_mass, grid_mom, dt: float,
                        gravity: Sequence[float] = (0.0, -9.8, 0.0), bc_layers: int = 1):
    """v_f = (m_f v_f) / m_f (Eq. 17) and v_s = (m_s v_s) / (m_s + m_f) (Eq. 20, the
    grid-summed mixture mass), each with the explicit update of ``grid_update``."""
    return np.stack([grid_update(grid, grid_mass[k], grid_mom[k], dt, gravity, bc_layers)
                     for k in (FLUID, SOLID)])


def mixture_g2p(grid: Grid, grid_vel, x, phase, n_modes: int, dt: float = 0.0, F=None):
    """G2P of each particle from its own phase's velocity field (grid_vel (2, 3, ...)),
    otherwise as ``g2p``; outputs in input order."""
    phase = np.asarray(phase)
    x = np.asarray(x, np.float32)
    P = x.shape[1]
    c_out = np.zeros((3, n_modes, P))
    x_out = np.zeros((3, P), np.float32)
    F_out = None if F is None else np.zeros((9, P))
    for k in (FLUID, SOLID):
        sel = np.flatnonzero(phase == k)
        Fk = None if F is None else np.asarray(F)[:, sel]
        ck, xk, fk = g2p(grid, grid_vel[k], x[:, sel], n_modes, dt, Fk)
        c_out[:, :, sel] = ck
        x_out[:, sel] = xk
        if F is not None:
            F_out[:, sel] = fk
    return c_out, x_out, F_out


# ---------------------------------------------------------------- one step

def step(grid: Grid, x, coeff, n_modes: int, dt: float, gravity=(0.0, -9.8, 0.0),
         bc_layers: int = 1, mass=None, uniform_mass: float = 1.0, F=None,
         sort: bool = True):
    """sort(x^n) -> P2G(x^n, c^n) -> grid update -> G2P(x^n) -> (c^{n+1}, x^{n+1}).

    When ``sort`` is set the outputs are in sorted order (output i belongs to
    input particle perm[i]), as the library writes them.
    Returns dict with keys perm, keys, grid_mass, grid_mom, grid_vel, coeff, x, F, mass.
    """
    x = np.asarray(x, np.float32)
    P = x.shape[1]
    if sort:
        keys, perm = sort_keys(grid, x)
    else:
        keys, perm = None, np.arange(P, dtype=np.int32)
    M, Q = p2g(grid, x, coeff, n_modes, mass, uniform_mass)
    v = grid_update(grid, M, Q, dt, gravity, bc_layers)
    xs = x[:, perm]
    Fs = None if F is None else np.asarray(F)[:, perm]
    c_out, x_out, F_out = g2p(grid, v, xs, n_modes, dt, Fs)
    m_out = None if mass is None else np.asarray(mass)[perm]
    return dict(perm=perm, keys=keys, grid_mass=M, grid_mom=Q, grid_vel=v,
                coeff=c_out, x=x_out, F=F_out, mass=m_out)


# ---------------------------------------------------------------- diagnostics

def normwise_rel_err(a, ref) -> float:
    """||a - ref||_2 / ||ref||_2 (0 if both vanish)."""
    a = np.asarray(a, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    den = np.linalg.norm(ref)
    num = np.linalg.norm(a - ref)
    if den == 0.0:
        return float(num)
    return float(num / den)
