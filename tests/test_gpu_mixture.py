"""Liquid and fabric particles on one grid (section 3.4, Eq. 15-20) on the GPU against the
FP64 oracle: fluid particles scatter at m_f into the fluid channels, fabric points at
m_s + m_f into the solid channels, and each particle is fitted from its own phase.
Bars: normwise 1e-5 (grid sums, velocities, coefficients), 1e-6 on F, positions within
2 float32 ulp, the per-particle arrays copied bit for bit."""
import json
import os
from fractions import Fraction as Fr

import numpy as np
import pytest
import torch

import workloads as W
from oracle import polypic_oracle as O
from tests.gpu_util import (TOL_NORMWISE, dev, host, note, oracle_grid, particles_touching, rel,
                            require_gpu, sample_nodes, ulp_ok)

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tiny_exact_mixture.json")


def _set(pp, g, s, nm, **kw):
    return pp.MixtureParticleSet(g, nm, dev(s.x), dev(s.coeff[:, :nm]), dev(s.phase, torch.int32),
                                 dev(s.mass_f), mass_s=dev(s.mass_s), F=dev(s.F), dt=s.dt,
                                 gravity=s.gravity, bc_layers=s.bc_layers, **kw)


def _mixed_random(seed, n=24, P=30_001):
    """Fluid and fabric particles scattered through the same cells."""
    rng = np.random.default_rng(seed)
    g = W.cubic_grid(n)
    x = ((3.0 + rng.random((3, P)) * (n - 2.0)) / n).astype(np.float32)
    c = np.zeros((3, 27, P), np.float32)
    c[:, 0] = rng.standard_normal((3, P))
    c[:, 1:] = 0.1 * rng.standard_normal((3, 26, P))
    phase = (rng.random(P) < 0.3).astype(np.int32)
    mass_s = np.where(phase == 1, 1.0 + rng.random(P), 0.0).astype(np.float32)
    mass_f = (0.5 * rng.random(P) + (phase == 0)).astype(np.float32)
    F = (np.eye(3).reshape(9, 1) + 0.01 * rng.standard_normal((9, P))).astype(np.float32)
    return W.MixtureScene("mixed_random", g, x, c, phase, mass_f, mass_s, F, dt=2e-3)


def _check_step(pp, s, nm):
    g = pp.grid_from_spec(s.grid)
    og = oracle_grid(g)
    ps = _set(pp, g, s, nm)
    ps.sort()
    ps.p2g()
    ps.grid_update()
    ps.g2p()
    torch.cuda.synchronize()
    assert ps.status_flags() == 0
    shp = (og.nz, og.ny, og.nx)
    M = host(ps.grid_mass).astype(np.float64).reshape((2,) + shp)
    Q = host(ps.grid_mom).astype(np.float64).reshape((2, 3) + shp)
    V = host(ps.grid_vel).astype(np.float64).reshape((2, 3) + shp)
    M_ref, Q_ref = O.mixture_p2g(og, s.x, s.coeff, nm, s.phase, s.mass_f, s.mass_s)
    for k in range(2):
        assert rel(M[k], M_ref[k]) <= TOL_NORMWISE, k
        assert rel(Q[k], Q_ref[k]) <= TOL_NORMWISE, k
    V_ref = O.mixture_grid_update(og, M, Q, s.dt, s.gravity, s.bc_layers)
    assert rel(V, V_ref) <= TOL_NORMWISE
    perm = host(ps.perm)
    _, pref = O.sort_keys(og, s.x)
    assert np.array_equal(perm, pref)
    c_ref, x_ref, F_ref = O.mixture_g2p(og, V, s.x[:, perm], s.phase[perm], nm, s.dt,
                                        s.F[:, perm])
    e_c = rel(host(ps.coeff_next).reshape(3, nm, s.P), c_ref)
    assert e_c <= TOL_NORMWISE
    assert ulp_ok(host(ps.x_next), x_ref, 2, og.nx * og.dx)
    assert rel(host(ps.F_next), F_ref) <= 1e-6
    assert np.array_equal(host(ps.phase_next), s.phase[perm])
    assert np.array_equal(host(ps.mass_f_next), s.mass_f[perm])
    assert np.array_equal(host(ps.mass_s_next), s.mass_s[perm])
    return e_c


@pytest.mark.parametrize("n_modes", [1, 4, 8, 27])
def test_mixture_step_mixed_cells(n_modes):
    """Fluid and fabric particles interleaved in the same cells (and bricks)."""
    pp = require_gpu()
    note(f"mixture step, mixed cells: n_modes={n_modes}")
    e = _check_step(pp, _mixed_random(1), n_modes)
    note(f"  coeff rel err {e:.2e}")


@pytest.mark.parametrize("n_modes", [4, 27])
def test_mixture_step_block_and_sheet(n_modes):
    """The liquid + fabric layout at test size: a fluid block above a fabric sheet, one grid."""
    pp = require_gpu()
    note(f"mixture step, block and sheet: n_modes={n_modes}")
    _check_step(pp, W.liquid_fabric_shared(0, n=32, side=100), n_modes)


@pytest.mark.parametrize("case_idx", range(4))
def test_mixture_exact_golden_fixture(case_idx):
    pp = require_gpu()
    with open(GOLDEN) as f:
        doc = json.load(f)
    case = doc["cases"][case_idx]
    nm = case["n_modes"]
    g = pp.make_grid(doc["nodes"], float(Fr(doc["dx"])))
    og = oracle_grid(g)
    x = np.array([[float(Fr(v)) for v in p] for p in doc["x"]], np.float32).T
    ms = np.array([float(Fr(v)) for v in doc["mass_s"]], np.float32)
    mf = np.array([float(Fr(v)) for v in doc["mass_f"]], np.float32)
    phase = np.array(doc["phase"], np.int32)
    cin = np.array([[[float(Fr(v)) for v in ca] for ca in c] for c in doc["coeff_in"]])
    cin = np.ascontiguousarray(np.transpose(cin, (1, 2, 0)).astype(np.float32))
    ps = pp.MixtureParticleSet(g, nm, dev(x), dev(cin[:, :nm]), dev(phase, torch.int32), dev(mf),
                               mass_s=dev(ms), dt=float(Fr(doc["dt"])),
                               gravity=[float(Fr(v)) for v in doc["gravity"]],
                               bc_layers=doc["bc_layers"])
    ps.p2g(use_perm=False)
    ps.grid_update()
    ps.g2p(use_perm=False)
    torch.cuda.synchronize()
    shp = (og.nz, og.ny, og.nx)
    M = host(ps.grid_mass).reshape((2,) + shp)
    Q = host(ps.grid_mom).reshape((2, 3) + shp)
    V = host(ps.grid_vel).reshape((2, 3) + shp)
    for k, ph in enumerate(case["phases"]):
        Me = np.zeros(shp)
        Qe = np.zeros((3,) + shp)
        Ve = np.zeros((3,) + shp)
        for nd, ms_, ps_, vs_ in zip(ph["nodes"], ph["grid_mass"], ph["grid_mom"],
                                     ph["grid_vel"]):
            ix, iy, iz = nd
            Me[iz, iy, ix] = float(Fr(ms_))
            for a in range(3):
                Qe[a, iz, iy, ix] = float(Fr(ps_[a]))
                Ve[a, iz, iy, ix] = float(Fr(vs_[a]))
        assert rel(M[k], Me) <= TOL_NORMWISE
        assert rel(Q[k], Qe) <= TOL_NORMWISE
        assert rel(V[k], Ve) <= TOL_NORMWISE
    ref = np.array([[[float(Fr(v)) for v in ca] for ca in cp] for cp in case["coeff"]])
    c = host(ps.coeff_next).reshape(3, nm, -1)
    assert rel(np.transpose(c, (2, 0, 1)), ref) <= TOL_NORMWISE


def test_mixture_unknown_phase_is_flagged_and_skipped():
    pp = require_gpu()
    s = _mixed_random(2, P=1000)
    s.phase[7] = 3
    g = pp.grid_from_spec(s.grid)
    ps = _set(pp, g, s, 4)
    ps.p2g(use_perm=False)
    torch.cuda.synchronize()
    assert ps.status_flags() & pp._lib.POLYPIC_FLAG_PHASE
    M = host(ps.grid_mass).reshape(2, -1).astype(np.float64)
    keep = np.arange(s.P) != 7
    fl = keep & (s.phase == 0)
    so = keep & (s.phase == 1)
    assert abs(M[0].sum() - s.mass_f[fl].astype(np.float64).sum()) < 1e-3
    assert abs(M[1].sum() - (s.mass_s[so] + s.mass_f[so]).astype(np.float64).sum()) < 1e-3


def test_mixture_full_size_sampled():
    """The liquid + fabric workload on one 260^3-node grid (16,777,216 fluid particles and
    1,000,000 fabric points, 27 modes) after two steps: the re-sort bit for bit, both
    channel sets at sampled nodes, their update there, and G2P at sampled slots."""
    pp = require_gpu()
    note("mixture full size: generating inputs")
    s = W.liquid_fabric_shared(0)
    g = pp.grid_from_spec(s.grid)
    og = oracle_grid(g)
    ps = _set(pp, g, s, 27, track_order=False)
    note(f"  P={s.P}: 2 steps")
    del s
    for _ in range(2):
        ps.step()
    x = host(ps.x).copy()
    c = host(ps.coeff).reshape(3, 27, ps.P).copy()
    phase, mf, ms = host(ps.phase).copy(), host(ps.mass_f).copy(), host(ps.mass_s).copy()
    ps.sort()
    ps.p2g()
    ps.grid_update()
    torch.cuda.synchronize()
    assert ps.status_flags() == 0
    _, pref = O.sort_keys(og, x)
    perm = host(ps.perm)
    assert np.array_equal(perm, pref)
    N = og.n_nodes
    M = host(ps.grid_mass).astype(np.float64).reshape(2, N)
    Q = host(ps.grid_mom).astype(np.float64).reshape(2, 3, N)
    V = host(ps.grid_vel).astype(np.float64).reshape(2, 3, N)
    for k in range(2):
        nodes = sample_nodes(M[k].reshape(og.nz, og.ny, og.nx), 300, seed=6 + k)
        sel = np.flatnonzero(phase == k)
        touch = sel[particles_touching(og, x[:, sel], nodes)]
        Mr, Qr = O.mixture_p2g(og, x[:, touch], c[:, :, touch], 27, phase[touch], mf[touch],
                               ms[touch])
        e_m = rel(M[k, nodes], Mr[k].ravel()[nodes])
        e_q = rel(Q[k][:, nodes], Qr[k].reshape(3, -1)[:, nodes])
        note(f"  phase {k}: {nodes.size} nodes, {touch.size} particles: {e_m:.2e} {e_q:.2e}")
        assert e_m <= TOL_NORMWISE and e_q <= TOL_NORMWISE
        shp = (og.nz, og.ny, og.nx)
        v_ref = O.grid_update(og, M[k].reshape(shp), Q[k].reshape((3,) + shp), ps.dt,
                              ps.gravity, ps.bc_layers).reshape(3, -1)
        assert rel(V[k][:, nodes], v_ref[:, nodes]) <= TOL_NORMWISE
    ps.g2p()
    torch.cuda.synchronize()
    rng = np.random.default_rng(8)
    fluid_slots = np.flatnonzero(phase[perm] == 0)
    solid_slots = np.flatnonzero(phase[perm] == 1)
    slots = np.sort(np.concatenate([rng.choice(fluid_slots, 4096, replace=False),
                                    rng.choice(solid_slots, 4096, replace=False)]))
    src = perm[slots]
    Vg = V.reshape((2, 3, og.nz, og.ny, og.nx))
    c_ref, x_ref, _ = O.mixture_g2p(og, Vg, x[:, src], phase[src], 27, ps.dt)
    e_c = rel(host(ps.coeff_next).reshape(3, 27, ps.P)[:, :, slots], c_ref)
    note(f"  G2P at {slots.size} slots (half fabric): {e_c:.2e}")
    assert e_c <= TOL_NORMWISE
    assert ulp_ok(host(ps.x_next)[:, slots], x_ref, 2, og.nx * og.dx)
