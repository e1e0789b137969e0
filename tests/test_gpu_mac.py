"""Staggered-grid (MAC) transfers on the GPU against the FP64 MAC oracle (oracle/mac.py).

Faces of component a sit at origin + (i + (1 - e_a)/2) dx, each with its own mass
(section 3, Table 1).  Bars as for the collocated grid: normwise 1e-5 on face masses,
momenta, velocities and coefficients, 1e-6 on F, positions within 2 float32 ulp,
the mass copy bit for bit.
"""
import json
import os
from fractions import Fraction as Fr

import numpy as np
import pytest
import torch

import workloads as W
from oracle import mac as MAC
from oracle import polypic_oracle as O
from tests.gpu_util import (TOL_NORMWISE, dev, host, note, oracle_grid, rel, require_gpu,
                            ulp_ok)

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tiny_exact_mac.json")


def _face_arrays(ps, og):
    shape = (3, og.nz, og.ny, og.nx)
    return (host(ps.grid_mass).astype(np.float64).reshape(shape),
            host(ps.grid_mom).astype(np.float64).reshape(shape),
            host(ps.grid_vel).astype(np.float64).reshape(shape))


def _check_step(pp, g, x, c, nm, mass=None, F=None, dt=1e-4, gravity=(0.0, -9.8, 0.0), bc=1,
                sort=True):
    og = oracle_grid(g)
    P = x.shape[1]
    ps = pp.MacParticleSet(g, nm, dev(x), dev(c[:, :nm]),
                           mass=None if mass is None else dev(mass),
                           F=None if F is None else dev(F), dt=dt, gravity=gravity,
                           bc_layers=bc)
    if sort:
        ps.sort()
    ps.p2g(use_perm=sort)
    ps.grid_update()
    ps.g2p(use_perm=sort)
    torch.cuda.synchronize()
    assert ps.status_flags() == 0
    M, Q, V = _face_arrays(ps, og)
    M_ref, Q_ref = MAC.p2g(og, x, c, nm, mass)
    for a in range(3):
        assert rel(M[a], M_ref[a]) <= TOL_NORMWISE, a
        assert rel(Q[a], Q_ref[a]) <= TOL_NORMWISE, a
    V_ref = MAC.grid_update(og, M, Q, dt, gravity, bc)   # teacher-forced with the device sums
    assert rel(V, V_ref) <= TOL_NORMWISE
    perm = host(ps.perm) if sort else np.arange(P)
    if sort:
        _, pref = O.sort_keys(og, x)
        assert np.array_equal(perm, pref)
    Fs = None if F is None else F[:, perm]
    c_ref, x_ref, F_ref = MAC.g2p(og, V, x[:, perm], nm, dt, Fs)
    c_out = host(ps.coeff_next).reshape(3, nm, P)
    e_c = rel(c_out, c_ref)
    assert e_c <= TOL_NORMWISE
    extent = og.nx * og.dx
    assert ulp_ok(host(ps.x_next), x_ref, 2, extent)
    if F is not None:
        assert rel(host(ps.F_next), F_ref) <= 1e-6
    if mass is not None:
        assert np.array_equal(host(ps.mass_next), mass[perm])
    return e_c


@pytest.mark.parametrize("n_modes", [1, 4, 8, 27])
def test_mac_step_matches_oracle_config0(n_modes):
    """The 32^3-cell parity case (32,768 particles, N(0,1) / N(0,0.1) coefficients) on a
    MAC grid, with random masses and F: sort, P2G, grid update, G2P + advection + F."""
    pp = require_gpu()
    s = W.config0(0)
    rng = np.random.default_rng(3)
    mass = (0.5 + rng.random(s.P)).astype(np.float32)
    F = (np.eye(3).reshape(9, 1) + 0.01 * rng.standard_normal((9, s.P))).astype(np.float32)
    note(f"mac step config0: n_modes={n_modes}")
    e = _check_step(pp, pp.grid_from_spec(s.grid), s.x, s.coeff, n_modes, mass=mass, F=F)
    note(f"  coeff rel err {e:.2e}")


@pytest.mark.parametrize("n_modes", [4, 27])
def test_mac_unsorted_and_ragged(n_modes):
    """Scattered particles in input order (every tile its own run: most go straight to HBM)
    and a count that is not a multiple of the workgroup."""
    pp = require_gpu()
    s = W.random_scene(5, 24, 10_001, mass_random=True)
    note(f"mac unsorted ragged: P={s.P} n_modes={n_modes}")
    g = pp.grid_from_spec(s.grid)
    _check_step(pp, g, s.x, s.coeff, n_modes, mass=s.mass, sort=False)
    _check_step(pp, g, s.x, s.coeff, n_modes, mass=s.mass, sort=True)


@pytest.mark.parametrize("case_idx", range(4))
def test_mac_exact_golden_fixture(case_idx):
    """The hand-placed particles of the exact-rational MAC fixture (staggered t = -1/2 on
    some axes, walls on): face sums, velocities, coefficients and positions."""
    pp = require_gpu()
    with open(GOLDEN) as f:
        doc = json.load(f)
    case = doc["cases"][case_idx]
    nm = case["n_modes"]
    nodes = doc["nodes"]
    dx = float(Fr(doc["dx"]))
    g = pp.make_grid(nodes, dx)
    og = oracle_grid(g)
    x = np.array([[float(Fr(v)) for v in p] for p in doc["x"]], np.float32).T
    mass = np.array([float(Fr(m)) for m in doc["mass"]], np.float32)
    cin = np.array([[[float(Fr(v)) for v in ca] for ca in c] for c in doc["coeff_in"]])
    cin = np.ascontiguousarray(np.transpose(cin, (1, 2, 0)).astype(np.float32))
    dt = float(Fr(doc["dt"]))
    grav = [float(Fr(v)) for v in doc["gravity"]]
    note(f"mac golden: n_modes={nm}")
    ps = pp.MacParticleSet(g, nm, dev(x), dev(cin[:, :nm]), mass=dev(mass), dt=dt, gravity=grav,
                           bc_layers=doc["bc_layers"])
    ps.p2g(use_perm=False)
    ps.grid_update()
    ps.g2p(use_perm=False)
    torch.cuda.synchronize()
    M, Q, V = _face_arrays(ps, og)
    Me = np.zeros_like(M)
    Qe = np.zeros_like(Q)
    Ve = np.zeros_like(V)
    for a, comp in enumerate(case["components"]):
        for fc, ms, qs, vs in zip(comp["faces"], comp["face_mass"], comp["face_mom"],
                                  comp["face_vel"]):
            ix, iy, iz = fc
            Me[a, iz, iy, ix] = float(Fr(ms))
            Qe[a, iz, iy, ix] = float(Fr(qs))
            Ve[a, iz, iy, ix] = float(Fr(vs))
    for a in range(3):
        assert rel(M[a], Me[a]) <= TOL_NORMWISE
        assert rel(Q[a], Qe[a]) <= TOL_NORMWISE
    assert rel(V, Ve) <= TOL_NORMWISE
    ref = np.array([[[float(Fr(v)) for v in ca] for ca in cp] for cp in case["coeff"]])
    c = host(ps.coeff_next).reshape(3, nm, -1)
    assert rel(np.transpose(c, (2, 0, 1)), ref) <= TOL_NORMWISE
    xref = np.array(case["x_out"], np.float32).T
    assert ulp_ok(host(ps.x_next), xref, 2, og.nx * og.dx)


def test_mac_out_of_range_and_empty():
    """A particle whose face stencils leave the arrays (u just below 1 on one axis) is
    flagged and skipped; P = 0 clears the face arrays."""
    pp = require_gpu()
    g = pp.make_grid((12, 12, 12), 1 / 8)
    below = float(np.nextafter(np.float32(1.0), np.float32(0.0)))
    x = np.array([[0.6, below / 8, 0.7], [0.6, 0.6, 0.7], [0.6, 0.6, 0.6]], np.float32)
    c = np.ones((3, 4, 3), np.float32)
    ps = pp.MacParticleSet(g, 4, dev(x), dev(c), dt=0.0, gravity=(0, 0, 0), bc_layers=0)
    ps.p2g(use_perm=False)
    torch.cuda.synchronize()
    assert ps.status_flags() & 1
    fm = host(ps.grid_mass).reshape(3, -1)
    assert np.allclose(fm.sum(axis=1), 2.0, atol=1e-6)   # the two in-range particles
    empty = pp.MacParticleSet(g, 4, dev(np.zeros((3, 0), np.float32)),
                              dev(np.zeros((3, 4, 0), np.float32)))
    empty.grid_mass.fill_(7.0)
    empty.grid_mom.fill_(7.0)
    empty.p2g(use_perm=False)
    torch.cuda.synchronize()
    assert float(empty.grid_mass.abs().max()) == 0.0 and float(empty.grid_mom.abs().max()) == 0.0


def test_mac_full_size_sampled():
    """The moving dam break (4,194,304 particles, 27 modes) on a MAC grid after three steps:
    the re-sort bit for bit, face sums at sampled faces of every component from the oracle
    run over the particles touching them, the update there, and G2P at sampled slots."""
    pp = require_gpu()
    s = W.config1_moving(0)
    g = pp.grid_from_spec(s.grid)
    og = oracle_grid(g)
    ps = pp.MacParticleSet(g, 27, dev(s.x), dev(s.coeff), dt=s.dt, gravity=s.gravity,
                           bc_layers=s.bc_layers, track_order=False)
    note(f"mac full size: P={s.P}, 3 steps")
    del s
    for _ in range(3):
        ps.step()
    x = host(ps.x).copy()
    c = host(ps.coeff).reshape(3, 27, ps.P).copy()
    ps.sort()
    ps.p2g()
    ps.grid_update()
    torch.cuda.synchronize()
    assert ps.status_flags() == 0
    _, pref = O.sort_keys(og, x)
    perm = host(ps.perm)
    assert np.array_equal(perm, pref)
    M, Q, V = _face_arrays(ps, og)
    rng = np.random.default_rng(4)
    for a in range(3):
        occ = np.flatnonzero(M[a].ravel() > 0)
        faces = np.unique(np.concatenate([rng.choice(occ, 150, replace=False),
                                          rng.integers(0, M[a].size, 50)]))
        iz, rem = np.divmod(faces, og.nx * og.ny)
        iy, ix = np.divmod(rem, og.nx)
        b, _ = MAC.face_stencil(og, x, a)
        flat_b = (b[2] * og.ny + b[1]) * og.nx + b[0]
        cand = []
        for dz in range(3):
            for dy in range(3):
                for dxx in range(3):
                    cand.append(((iz - dz) * og.ny + (iy - dy)) * og.nx + (ix - dxx))
        touch = np.flatnonzero(np.isin(flat_b, np.concatenate(cand)))
        M_ref, Q_ref = MAC.p2g(og, x[:, touch], c[:, :, touch], 27)
        e_m = rel(M[a].ravel()[faces], M_ref[a].ravel()[faces])
        e_q = rel(Q[a].ravel()[faces], Q_ref[a].ravel()[faces])
        note(f"  component {a}: {faces.size} faces, {touch.size} particles: {e_m:.2e} {e_q:.2e}")
        assert e_m <= TOL_NORMWISE and e_q <= TOL_NORMWISE
    V_ref = MAC.grid_update(og, M, Q, ps.dt, ps.gravity, ps.bc_layers)
    assert rel(V, V_ref) <= TOL_NORMWISE
    ps.g2p()
    torch.cuda.synchronize()
    slots = np.sort(rng.choice(ps.P, 8192, replace=False))
    c_ref, x_ref, _ = MAC.g2p(og, V, x[:, perm[slots]], 27, ps.dt)
    c_out = host(ps.coeff_next).reshape(3, 27, ps.P)[:, :, slots]
    e_c = rel(c_out, c_ref)
    note(f"  G2P at {slots.size} slots: {e_c:.2e}")
    assert e_c <= TOL_NORMWISE
    assert ulp_ok(host(ps.x_next)[:, slots], x_ref, 2, og.nx * og.dx)
