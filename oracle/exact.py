"""Exact-rational brute force of the PolyPIC transfers -- TEST INFRASTRUCTURE ONLY.

An independent second statement of the transfers in ``fractions.Fraction``
arithmetic for tiny inputs (a handful of particles on a small grid).  It
shares no code with ``polypic_oracle`` and makes none of its simplifications:

* weights are the quadratic B-spline evaluated piecewise (section 3.1);
* modes are the monomial products of Eq. 11 with the quadratic factor
  replaced by Eq. 14 (read as g(z) = z^2 - a z - 1/4 in units of dx, with
  a = t (1 - 4 t^2) and t the particle's offset from its nearest node);
* G2P solves the weighted least-squares problem of section 3.3 through its
  full normal equations (Gaussian elimination, no orthogonality assumed);
  where some weights vanish (t = -1/2) and the fit is not unique, the
  27-mode case is the interpolation E c = v (E is invertible there), and the
  1/4/8-mode cases are still unique because they hold no quadratic factor.

Inputs must be dyadic so that the float32 stencil formula is exact; the
functions check this.
"""
from __future__ import annotations

import itertools
from fractions import Fraction as Fr
from typing import Dict, List, Sequence, Tuple

import numpy as np

MODE_EXPONENTS = (
    (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, 0, 1), (0, 1, 1), (1, 1, 1),
    (2, 0, 0), (0, 2, 0), (0, 0, 2), (2, 1, 0), (2, 0, 1), (1, 2, 0), (0, 2, 1), (1, 0, 2),
    (0, 1, 2), (2, 1, 1), (1, 2, 1), (1, 1, 2), (2, 2, 0), (2, 0, 2), (0, 2, 2), (2, 2, 1),
    (2, 1, 2), (1, 2, 2), (2, 2, 2),
)

Node = Tuple[int, int, int]


def bspline2(d: Fr) -> Fr:
    """Quadratic B-spline, piecewise."""
    a = abs(d)
    if a < Fr(1, 2):
        return Fr(3, 4) - a * a
    if a < Fr(3, 2):
        return (Fr(3, 2) - a) ** 2 / 2
    return Fr(0)


def to_fraction_exact(v) -> Fr:
    """Exact rational value of a float (float32 values convert exactly)."""
    return Fr(float(v))


def stencil(u: Fr) -> Tuple[int, Fr]:
    """Base node b = floor(u - 1/2) and t = u - b - 1."""
    b = (u - Fr(1, 2)).__floor__()
    return b, u - b - 1


def ghat(z: Fr, t: Fr) -> Fr:
    a = t * (1 - 4 * t * t)
    return z * z - a * z - Fr(1, 4)


def mode_value(k: int, z: Fr, t: Fr) -> Fr:
    if k == 0:
        return Fr(1)
    if k == 1:
        return z
    return ghat(z, t)


class ParticleStencil:
    """Exact stencil data of one particle: base node, per-axis t, node weights, modes.

    ``shift`` (in units of dx, per axis) moves the lattice the stencil lives on: the
    faces of a staggered grid sit at origin + (i + shift) dx."""

    def __init__(self, x: Sequence[Fr], origin: Sequence[Fr], inv_dx: Fr,
                 shift: Sequence[Fr] = (Fr(0), Fr(0), Fr(0))):
        self.u = [(x[a] - origin[a]) * inv_dx - shift[a] for a in range(3)]
        bt = [stencil(u) for u in self.u]
        self.b = [p[0] for p in bt]
        self.t = [p[1] for p in bt]

    def nodes(self) -> List[Tuple[Node, Tuple[int, int, int]]]:
        out = []
        for j in itertools.product(range(3), repeat=3):
            out.append(((self.b[0] + j[0], self.b[1] + j[1], self.b[2] + j[2]), j))
        return out

    def zhat(self, a: int, j: int) -> Fr:
        return Fr(self.b[a] + j) - self.u[a]

    def weight(self, j) -> Fr:
        w = Fr(1)
        for a in range(3):
            w *= bspline2(self.zhat(a, j[a]))
        return w

    def mode(self, r: int, j) -> Fr:
        s = Fr(1)
        for a in range(3):
            s *= mode_value(MODE_EXPONENTS[r][a], self.zhat(a, j[a]), self.t[a])
        return s


def p2g(xs, origin, inv_dx, coeffs, masses, n_modes) -> Dict[Node, Tuple[Fr, List[Fr]]]:
    """Exact grid mass and momentum: dict node -> (m, [p_x, p_y, p_z])."""
    grid: Dict[Node, Tuple[Fr, List[Fr]]] = {}
    for x, c, m in zip(xs, coeffs, masses):
        ps = ParticleStencil(x, origin, inv_dx)
        for node, j in ps.nodes():
            W = ps.weight(j)
            mi, pi = grid.get(node, (Fr(0), [Fr(0)] * 3))
            mi = mi + m * W
            pi = list(pi)
            for a in range(3):
                val = sum((c[a][r] * ps.mode(r, j) for r in range(n_modes)), Fr(0))
                pi[a] += m * W * val
            grid[node] = (mi, pi)
    return grid


def grid_update(grid, dims, dt: Fr, gravity: Sequence[Fr], bc_layers: int):
    """Exact v = p/m + dt g on nodes with m > 0, then separating slip walls."""
    out: Dict[Node, List[Fr]] = {}
    for node, (m, p) in grid.items():
        if m > 0:
            v = [p[a] / m + dt * gravity[a] for a in range(3)]
        else:
            v = [Fr(0)] * 3
        if bc_layers > 0:
            for a in range(3):
                if node[a] <= 1 + bc_layers and v[a] < 0:
                    v[a] = Fr(0)
                if node[a] >= dims[a] - 1 - bc_layers and v[a] > 0:
                    v[a] = Fr(0)
        out[node] = v
    return out


def solve(A: List[List[Fr]], rhs: List[List[Fr]]) -> List[List[Fr]]:
    """Gauss-Jordan elimination with row pivoting; A n x n, rhs n x k. Raises if singular."""
    n = len(A)
    k = len(rhs[0])
    M = [list(A[i]) + list(rhs[i]) for i in range(n)]
    for col in range(n):
        piv = next((r for r in range(col, n) if M[r][col] != 0), None)
        if piv is None:
            raise ZeroDivisionError("singular system")
        M[col], M[piv] = M[piv], M[col]
        inv = 1 / M[col][col]
        M[col] = [v * inv for v in M[col]]
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col]
                M[r] = [vr - f * vc for vr, vc in zip(M[r], M[col])]
    return [row[n:n + k] for row in M]


def g2p_particle(ps: ParticleStencil, vel: Dict[Node, List[Fr]], n_modes: int) -> List[List[Fr]]:
    """Weighted least-squares fit of the first n_modes modes to the 27 node velocities.

    Returns c[a][r].  Uses the normal equations S^T W S c = S^T W v unless the
    weights vanish somewhere and n_modes == 27, where the fit is the
    interpolation S c = v.
    """
    rows = ps.nodes()
    S = [[ps.mode(r, j) for r in range(n_modes)] for _, j in rows]
    W = [ps.weight(j) for _, j in rows]
    V = [[vel.get(node, [Fr(0)] * 3)[a] for a in range(3)] for node, _ in rows]
    degenerate = any(w == 0 for w in W)
    if degenerate and n_modes == 27:
        sol = solve(S, V)
    else:
        A = [[sum((W[i] * S[i][r] * S[i][s] for i in range(27)), Fr(0)) for s in range(n_modes)]
             for r in range(n_modes)]
        rhs = [[sum((W[i] * S[i][r] * V[i][a] for i in range(27)), Fr(0)) for a in range(3)]
               for r in range(n_modes)]
        sol = solve(A, rhs)
    return [[sol[r][a] for r in range(n_modes)] for a in range(3)]


def g2p(xs, origin, inv_dx, vel, n_modes):
    return [g2p_particle(ParticleStencil(x, origin, inv_dx), vel, n_modes) for x in xs]


def float32_round(v: Fr) -> np.float32:
    """Round an exact rational to the nearest float32 (ties to even)."""
    f64 = float(v)                 # correctly rounded to float64
    f32 = np.float32(f64)
    # double rounding can only matter at exact float32 ties; resolve them exactly
    cand = [np.nextafter(f32, np.float32(-np.inf)), f32, np.nextafter(f32, np.float32(np.inf))]
    best = min(cand, key=lambda c: (abs(Fr(float(c)) - v),
                                    int(np.frombuffer(np.float32(c).tobytes(), np.uint32)[0]) & 1))
    return np.float32(best)


# ---------------------------------------------------------------- staggered (MAC) grid
# Section 3 applies the transfers on marker-and-cell grids: component alpha lives on
# the faces at origin + (i + (1 - e_alpha)/2) dx, each with its own mass.  Every
# component is a scalar transfer on its own shifted lattice.

def face_shift(alpha: int) -> Tuple[Fr, Fr, Fr]:
    return tuple(Fr(0) if a == alpha else Fr(1, 2) for a in range(3))


def mac_p2g(xs, origin, inv_dx, coeffs, masses, n_modes) -> List[Dict[Node, Tuple[Fr, Fr]]]:
    """Exact face mass and momentum of each component: [dict face -> (m, p)] * 3."""
    out = []
    for alpha in range(3):
        grid: Dict[Node, Tuple[Fr, Fr]] = {}
        for x, c, m in zip(xs, coeffs, masses):
            ps = ParticleStencil(x, origin, inv_dx, face_shift(alpha))
            for node, j in ps.nodes():
                W = ps.weight(j)
                mi, pi = grid.get(node, (Fr(0), Fr(0)))
                val = sum((c[alpha][r] * ps.mode(r, j) for r in range(n_modes)), Fr(0))
                grid[node] = (mi + m * W, pi + m * W * val)
        out.append(grid)
    return out


def mac_grid_update(grids, dims, dt: Fr, gravity: Sequence[Fr], bc_layers: int):
    """Exact v = p/m + dt g_alpha on faces with m > 0, then the walls of axis alpha."""
    out = []
    for alpha, grid in enumerate(grids):
        vel: Dict[Node, Fr] = {}
        for node, (m, p) in grid.items():
            v = p / m + dt * gravity[alpha] if m > 0 else Fr(0)
            if bc_layers > 0:
                if node[alpha] <= 1 + bc_layers and v < 0:
                    v = Fr(0)
                if node[alpha] >= dims[alpha] - 1 - bc_layers and v > 0:
                    v = Fr(0)
            vel[node] = v
        out.append(vel)
    return out


def mac_g2p(xs, origin, inv_dx, vels, n_modes):
    """Per particle c[alpha][r]: the least-squares fit of component alpha over its own
    face stencil (as g2p_particle, one component at a time)."""
    res = []
    for x in xs:
        c = []
        for alpha in range(3):
            ps = ParticleStencil(x, origin, inv_dx, face_shift(alpha))
            v3 = {node: [v, v, v] for node, v in vels[alpha].items()}
            c.append(g2p_particle(ps, v3, n_modes)[alpha])
        res.append(c)
    return res


# ---------------------------------------------------------------- affine back-map (Eq. 12-13)

def inverse3(A: List[List[Fr]]) -> List[List[Fr]]:
    """Exact inverse of a 3 x 3 matrix (Gauss-Jordan on [A | I])."""
    eye = [[Fr(int(i == j)) for j in range(3)] for i in range(3)]
    return solve(A, eye)


def p2g_affine(xs, xs_fit, origin, inv_dx, coeffs, masses, n_modes, dt: Fr, dx: Fr):
    """Exact grid mass and momentum with the modes evaluated at
    z' = (I + dt C)^-1 (x_i - x_p) / dx (Eq. 12 applied in Eq. 13), C_ab = c_{a,1+b} / dx,
    and the quadratic factor g(z) = z^2 - a z - 1/4 with a from the particle's offset at
    x_fit (the position where its coefficients were fitted)."""
    grid: Dict[Node, Tuple[Fr, List[Fr]]] = {}
    for x, xf, c, m in zip(xs, xs_fit, coeffs, masses):
        ps = ParticleStencil(x, origin, inv_dx)
        t_fit = ParticleStencil(xf, origin, inv_dx).t
        A = [[Fr(int(a == b)) for b in range(3)] for a in range(3)]
        if n_modes >= 4:
            for a in range(3):
                for b in range(3):
                    A[a][b] += dt * c[a][1 + b] / dx
        Ainv = inverse3(A)
        for node, j in ps.nodes():
            W = ps.weight(j)
            z = [ps.zhat(a, j[a]) for a in range(3)]
            zp = [sum((Ainv[a][b] * z[b] for b in range(3)), Fr(0)) for a in range(3)]
            mi, pi = grid.get(node, (Fr(0), [Fr(0)] * 3))
            pi = list(pi)
            for al in range(3):
                val = Fr(0)
                for r in range(n_modes):
                    s = Fr(1)
                    for a in range(3):
                        s *= mode_value(MODE_EXPONENTS[r][a], zp[a], t_fit[a])
                    val += c[al][r] * s
                pi[al] += m * W * val
            grid[node] = (mi + m * W, pi)
    return grid
