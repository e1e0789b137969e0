"""Writes tests/golden/tiny_exact.json: exact-rational results of one transfer step.

The stored values are computed only by ``oracle/exact.py`` (exact rational
arithmetic, normal-equation least squares, no orthogonality assumed).  The
paper prints no worked numeric example, so these tiny hand-placed cases stand
in for one; they cover the stencil offsets t = -1/2 (degenerate weights),
t = 0 and t = 1/2 - 2^-20, unequal masses, and all four mode counts.

Run:  python tests/golden/make_golden.py   (writes tiny_exact.json, tiny_exact_mac.json,
      tiny_exact_affine.json and tiny_exact_mixture.json)
"""
from __future__ import annotations

import json
import os
import sys
from fractions import Fraction as Fr

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import exact  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiny_exact.json")
OUT_MAC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiny_exact_mac.json")
OUT_AFFINE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiny_exact_affine.json")
OUT_MIXTURE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiny_exact_mixture.json")

# grid: 4 cells per axis -> 8 nodes per axis, dx = 1/4, origin 0, domain [0.5, 1.5)
NODES = (8, 8, 8)
DX = Fr(1, 4)
INV_DX = Fr(4)
ORIGIN = (Fr(0), Fr(0), Fr(0))
DT = Fr(1, 1024)
GRAVITY = (Fr(0), Fr(-49, 5), Fr(0))
BC_LAYERS = 1


def particles():
    """Six particles, positions given by their grid coordinate u (x = u * dx)."""
    tiny = Fr(1, 2 ** 20)
    us = [
        (Fr(7, 2), Fr(4), Fr(9, 2) - tiny),          # t = (-1/2, 0, 1/2 - 2^-20)
        (Fr(4) + Fr(3, 16), Fr(3) + Fr(5, 8), Fr(4) - Fr(1, 32)),
        (Fr(3) + Fr(1, 2) + Fr(1, 64), Fr(7, 2), Fr(4) + Fr(7, 32)),   # t_y = -1/2
        (Fr(4) + Fr(11, 32), Fr(4) + Fr(5, 16), Fr(3) + Fr(9, 16)),
        (Fr(5) + Fr(1, 4), Fr(4) + Fr(15, 32), Fr(4) + Fr(3, 8)),
        (Fr(2) + Fr(3, 8), Fr(5) + Fr(1, 2) - tiny, Fr(3) + Fr(1, 2)),  # near low x wall
    ]
    xs = [tuple(u * DX for u in p) for p in us]
    masses = [Fr(1), Fr(3, 2), Fr(1), Fr(5, 4), Fr(1), Fr(3, 4)]
    # dyadic coefficients: c[a][r] = small integers / 16, deterministic pattern
    rng = np.random.default_rng(7)
    coeffs = []
    for _ in xs:
        c = [[Fr(int(v), 16) for v in rng.integers(-24, 25, size=27)] for _ in range(3)]
        coeffs.append(c)
    return xs, masses, coeffs


def fstr(v: Fr) -> str:
    return f"{v.numerator}/{v.denominator}"


def main():
    xs, masses, coeffs = particles()
    for x in xs:
        for a in range(3):
            assert Fr(float(np.float32(float(x[a])))) == x[a], "positions must be float32-exact"
    cases = []
    lo = [ORIGIN[a] + 2 * DX for a in range(3)]
    for n_modes in (1, 4, 8, 27):
        grid = exact.p2g(xs, ORIGIN, INV_DX, coeffs, masses, n_modes)
        vel = exact.grid_update(grid, NODES, DT, GRAVITY, BC_LAYERS)
        cs = exact.g2p(xs, ORIGIN, INV_DX, vel, n_modes)
        x_out = []
        for x, c in zip(xs, cs):
            row = []
            for a in range(3):
                xn = exact.float32_round(x[a] + DT * c[a][0])
                top = np.float32(float(ORIGIN[a] + (NODES[a] - 2) * DX))
                hi = np.nextafter(top, np.float32(-np.inf))
                xn = min(max(xn, np.float32(float(lo[a]))), hi)
                row.append(float(xn))
            x_out.append(row)
        nodes = sorted(grid.keys())
        cases.append(dict(
            n_modes=n_modes,
            nodes=[list(nd) for nd in nodes],
            grid_mass=[fstr(grid[nd][0]) for nd in nodes],
            grid_mom=[[fstr(v) for v in grid[nd][1]] for nd in nodes],
            grid_vel=[[fstr(v) for v in vel[nd]] for nd in nodes],
            coeff=[[[fstr(v) for v in c[a]] for a in range(3)] for c in cs],
            x_out=x_out,
        ))
    doc = dict(
        description="Exact-rational P2G -> grid update -> G2P on 6 hand-placed particles "
                    "(written by tests/golden/make_golden.py from oracle/exact.py)",
        nodes=list(NODES), dx=fstr(DX), inv_dx=fstr(INV_DX), origin=[fstr(o) for o in ORIGIN],
        dt=fstr(DT), gravity=[fstr(g) for g in GRAVITY], bc_layers=BC_LAYERS,
        x=[[fstr(v) for v in x] for x in xs],
        mass=[fstr(m) for m in masses],
        coeff_in=[[[fstr(v) for v in c[a]] for a in range(3)] for c in coeffs],
        cases=cases,
    )
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", OUT)
    write_mac(xs, masses, coeffs)
    write_affine(xs, masses, coeffs)
    write_mixture(xs, masses, coeffs)


def write_mixture(xs, masses, coeffs):
    """Liquid and fabric particles on one grid (section 3.4): particles 1, 3 and 4 are
    solid (fabric) with solid mass m_s and absorbed fluid m_f, the others fluid with mass
    m_f.  The fluid channels get the fluid particles at m_f (Eq. 15-16), the solid
    channels the solid ones at m_s + m_f (Eq. 18-19); each phase's velocity (Eq. 17, 20)
    is fitted back only by its own particles."""
    phase = [0, 1, 0, 1, 1, 0]
    mass_f = [Fr(3, 4), Fr(1, 4), Fr(5, 4), Fr(0), Fr(3, 8), Fr(1)]
    mass_s = masses
    cases = []
    for n_modes in (1, 4, 8, 27):
        per = []
        for k in (0, 1):
            sel = [p for p in range(len(xs)) if phase[p] == k]
            m = [mass_f[p] if k == 0 else mass_s[p] + mass_f[p] for p in sel]
            grid = exact.p2g([xs[p] for p in sel], ORIGIN, INV_DX, [coeffs[p] for p in sel], m,
                             n_modes)
            vel = exact.grid_update(grid, NODES, DT, GRAVITY, BC_LAYERS)
            per.append((grid, vel))
        cs = [exact.g2p([x], ORIGIN, INV_DX, per[phase[p]][1], n_modes)[0]
              for p, x in enumerate(xs)]
        phases = []
        for k in (0, 1):
            grid, vel = per[k]
            nodes = sorted(grid.keys())
            phases.append(dict(
                nodes=[list(nd) for nd in nodes],
                grid_mass=[fstr(grid[nd][0]) for nd in nodes],
                grid_mom=[[fstr(v) for v in grid[nd][1]] for nd in nodes],
                grid_vel=[[fstr(v) for v in vel[nd]] for nd in nodes],
            ))
        cases.append(dict(n_modes=n_modes, phases=phases,
                          coeff=[[[fstr(v) for v in c[a]] for a in range(3)] for c in cs]))
    doc = dict(
        description="Exact-rational shared-grid liquid-fabric transfers: P2G of each phase "
                    "into its own channels, grid update, G2P of each particle from its "
                    "phase's velocity (written by tests/golden/make_golden.py from "
                    "oracle/exact.py)",
        nodes=list(NODES), dx=fstr(DX), inv_dx=fstr(INV_DX), origin=[fstr(o) for o in ORIGIN],
        dt=fstr(DT), gravity=[fstr(g) for g in GRAVITY], bc_layers=BC_LAYERS,
        x=[[fstr(v) for v in x] for x in xs],
        phase=phase,
        mass_s=[fstr(m) for m in mass_s],
        mass_f=[fstr(m) for m in mass_f],
        coeff_in=[[[fstr(v) for v in c[a]] for a in range(3)] for c in coeffs],
        cases=cases,
    )
    with open(OUT_MIXTURE, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", OUT_MIXTURE)


def write_affine(xs, masses, coeffs):
    """P2G with the affine back-map of Eq. 12 on the same particles: each particle's
    coefficients are taken as fitted at a nearby earlier position x_fit (a few
    1/64-cell steps away, one of them across a cell switch), with a time step large
    enough that I + dt C is far from the identity."""
    shifts = [(Fr(1, 64), Fr(-3, 64), Fr(2, 64)), (Fr(-5, 64), Fr(1, 64), Fr(0)),
              (Fr(0), Fr(3, 64), Fr(-1, 64)), (Fr(2, 64), Fr(2, 64), Fr(2, 64)),
              (Fr(-1, 64), Fr(0), Fr(9, 64)), (Fr(4, 64), Fr(-2, 64), Fr(1, 64))]
    xs_fit = [tuple(x[a] + shifts[k][a] * DX for a in range(3)) for k, x in enumerate(xs)]
    dt = Fr(1, 64)
    cases = []
    for n_modes in (1, 4, 8, 27):
        grid = exact.p2g_affine(xs, xs_fit, ORIGIN, INV_DX, coeffs, masses, n_modes, dt, DX)
        nodes = sorted(grid.keys())
        cases.append(dict(
            n_modes=n_modes,
            nodes=[list(nd) for nd in nodes],
            grid_mass=[fstr(grid[nd][0]) for nd in nodes],
            grid_mom=[[fstr(v) for v in grid[nd][1]] for nd in nodes],
        ))
    doc = dict(
        description="Exact-rational P2G with the affine back-map of Eq. 12 (modes at "
                    "(I + dt C)^-1 (x_i - x_p) / dx, quadratic factor of the fitting position) "
                    "on 6 hand-placed particles (written by tests/golden/make_golden.py from "
                    "oracle/exact.py)",
        nodes=list(NODES), dx=fstr(DX), inv_dx=fstr(INV_DX), origin=[fstr(o) for o in ORIGIN],
        dt=fstr(dt),
        x=[[fstr(v) for v in x] for x in xs],
        x_fit=[[fstr(v) for v in x] for x in xs_fit],
        mass=[fstr(m) for m in masses],
        coeff_in=[[[fstr(v) for v in c[a]] for a in range(3)] for c in coeffs],
        cases=cases,
    )
    with open(OUT_AFFINE, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", OUT_AFFINE)


def write_mac(xs, masses, coeffs):
    """The same particles on a staggered (MAC) grid: component alpha on the faces at
    origin + (i + (1 - e_alpha)/2) dx, each face with its own mass (section 3).  The
    staggered offsets t = frac(u) - 1/2 include -1/2 (u integral) on some axes."""
    cases = []
    lo = [ORIGIN[a] + 2 * DX for a in range(3)]
    for n_modes in (1, 4, 8, 27):
        grids = exact.mac_p2g(xs, ORIGIN, INV_DX, coeffs, masses, n_modes)
        vels = exact.mac_grid_update(grids, NODES, DT, GRAVITY, BC_LAYERS)
        cs = exact.mac_g2p(xs, ORIGIN, INV_DX, vels, n_modes)
        x_out = []
        for x, c in zip(xs, cs):
            row = []
            for a in range(3):
                xn = exact.float32_round(x[a] + DT * c[a][0])
                top = np.float32(float(ORIGIN[a] + (NODES[a] - 2) * DX))
                hi = np.nextafter(top, np.float32(-np.inf))
                xn = min(max(xn, np.float32(float(lo[a]))), hi)
                row.append(float(xn))
            x_out.append(row)
        comps = []
        for alpha in range(3):
            faces = sorted(grids[alpha].keys())
            comps.append(dict(
                faces=[list(f) for f in faces],
                face_mass=[fstr(grids[alpha][f][0]) for f in faces],
                face_mom=[fstr(grids[alpha][f][1]) for f in faces],
                face_vel=[fstr(vels[alpha][f]) for f in faces],
            ))
        cases.append(dict(
            n_modes=n_modes,
            components=comps,
            coeff=[[[fstr(v) for v in c[a]] for a in range(3)] for c in cs],
            x_out=x_out,
        ))
    doc = dict(
        description="Exact-rational P2G -> grid update -> G2P on a staggered (MAC) grid, "
                    "6 hand-placed particles (written by tests/golden/make_golden.py from "
                    "oracle/exact.py)",
        nodes=list(NODES), dx=fstr(DX), inv_dx=fstr(INV_DX), origin=[fstr(o) for o in ORIGIN],
        dt=fstr(DT), gravity=[fstr(g) for g in GRAVITY], bc_layers=BC_LAYERS,
        x=[[fstr(v) for v in x] for x in xs],
        mass=[fstr(m) for m in masses],
        coeff_in=[[[fstr(v) for v in c[a]] for a in range(3)] for c in coeffs],
        cases=cases,
    )
    with open(OUT_MAC, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", OUT_MAC)


if __name__ == "__main__":
    main()
