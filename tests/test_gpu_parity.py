"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bars: sort keys and permutation bit-exact; grid mass, grid momentum and
particle coefficients within 1e-5 normwise relative error; positions within
2 float32 ulps of the domain extent.  Inputs are the seeded workloads of the
`workloads` package (single-step 32^3 case, random and ragged scenes).
"""
import json
import os
from fractions import Fraction as Fr

import numpy as np
import pytest
import torch

import workloads as W
from oracle import polypic_oracle as O
from tests.gpu_util import p2g_config
from tests.gpu_util import (TOL_NORMWISE, dev, host, note, oracle_grid, rel, require_gpu,
                            ulp_ok)

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tiny_exact.json")


def particle_set(scene, n_modes, dt=None, gravity=None, bc_layers=None, with_mass=True,
                 **kw):
    pp = require_gpu()
    g = pp.grid_from_spec(scene.grid)
    ps = pp.ParticleSet(
        g, n_modes, dev(scene.x), dev(scene.coeff[:, :n_modes]),
        mass=dev(scene.mass) if (with_mass and scene.mass is not None) else None,
        uniform_mass=scene.uniform_mass,
        F=dev(scene.F) if scene.F is not None else None,
        dt=scene.dt if dt is None else dt,
        gravity=scene.gravity if gravity is None else gravity,
        bc_layers=scene.bc_layers if bc_layers is None else bc_layers, **kw)
    return pp, g, ps


def check_grid_of_state(ps, og, n_modes, mass=None, uniform_mass=1.0):
    """After a fused step the grid holds the P2G of the new state: compare it with the
    oracle's P2G of the state the device wrote (teacher-forced positions and coefficients)."""
    P = ps.P
    M_ref, Q_ref = O.p2g(og, host(ps.x), host(ps.coeff).reshape(3, n_modes, P), n_modes,
                         None if mass is None else host(mass), uniform_mass)
    assert rel(host(ps.grid_mass).reshape(M_ref.shape), M_ref) <= TOL_NORMWISE
    assert rel(host(ps.grid_mom).reshape(Q_ref.shape), Q_ref) <= TOL_NORMWISE


# ---------------------------------------------------------------- sort

@pytest.mark.parametrize("case", ["config0", "random_ragged", "tiny"])
def test_sort_bit_exact(case):
    if case == "config0":
        s = W.config0(0)
    elif case == "random_ragged":
        s = W.random_scene(3, 40, 20000 + 37)
    else:
        s = W.random_scene(4, 8, 5)
    note(f"sort parity: {case} P={s.P}")
    pp, g, ps = particle_set(s, 1)
    ps.sort()
    torch.cuda.synchronize()
    keys_ref, perm_ref = O.sort_keys(oracle_grid(g), s.x)
    assert np.array_equal(host(ps.keys).view(np.uint32), keys_ref)
    assert np.array_equal(host(ps.perm), perm_ref)
    assert ps.status_flags() == 0


def test_sort_presorted_and_reversed():
    """Already-sorted input gives the identity; duplicated keys keep input order."""
    s = W.config0(1)
    g0 = O.grid_from_spec(s.grid)
    _, perm = O.sort_keys(g0, s.x)
    xs = s.x[:, perm]
    pp, g, ps = particle_set(W.Scene("sorted", s.grid, xs, s.coeff[:, :, perm], None), 1)
    ps.sort()
    torch.cuda.synchronize()
    assert np.array_equal(host(ps.perm), np.arange(s.P, dtype=np.int32))
    xr = xs[:, ::-1].copy()
    pp, g, ps = particle_set(W.Scene("rev", s.grid, xr, s.coeff[:, :, ::-1].copy(), None), 1)
    ps.sort()
    torch.cuda.synchronize()
    _, perm_ref = O.sort_keys(g0, xr)
    assert np.array_equal(host(ps.perm), perm_ref)


# ---------------------------------------------------------------- P2G

@pytest.mark.parametrize("n_modes", O.ALLOWED_N_MODES)
@pytest.mark.parametrize("path", ["cells", "bricks", "unsorted"])
def test_p2g_parity(n_modes, path):
    """P2G on all three paths: cell gather (sorted keys), brick scatter in sorted
    order (perm only), brick scatter in input order."""
    s = W.config0(0)
    note(f"p2g parity: config0 P={s.P} n_modes={n_modes} path={path}")
    pp, g, ps = particle_set(s, n_modes)
    if path != "unsorted":
        ps.sort()
    with p2g_config(pp, n_modes, pp.POLYPIC_P2G_CELLS if path == "cells" else pp.POLYPIC_P2G_BRICKS):
        ps.p2g(use_perm=(path != "unsorted"), use_keys=(path == "cells"))
        torch.cuda.synchronize()
    M_ref, Q_ref = O.p2g(oracle_grid(g), s.x, s.coeff, n_modes)
    M = host(ps.grid_mass).reshape(M_ref.shape)
    Q = host(ps.grid_mom).reshape(Q_ref.shape)
    em, ep = rel(M, M_ref), rel(Q, Q_ref)
    note(f"  mass {em:.2e}  momentum {ep:.2e}")
    assert em <= TOL_NORMWISE and ep <= TOL_NORMWISE
    assert ps.status_flags() == 0


def test_p2g_random_masses_and_accumulate():
    """Per-particle masses (Eq. 18's m_s + m_f) and accumulate = 1 adding a second and
    third pass (cell-gather and brick paths)."""
    s = W.random_scene(5, 24, 9001, mass_random=True)
    note(f"p2g mass/accumulate: P={s.P}")
    pp, g, ps = particle_set(s, 27)
    ps.sort()
    ps.p2g()
    pp.polypic_p2g(g, 27, ps.x, ps.coeff, ps.grid_mass, ps.grid_mom, mass=ps.mass,
                   perm=ps.perm, keys_sorted=ps.keys, ws=ps.p2g_ws, accumulate=True)
    pp.polypic_p2g(g, 27, ps.x, ps.coeff, ps.grid_mass, ps.grid_mom, mass=ps.mass,
                   perm=ps.perm, accumulate=True)
    torch.cuda.synchronize()
    M_ref, Q_ref = O.p2g(oracle_grid(g), s.x, s.coeff, 27, s.mass)
    assert rel(host(ps.grid_mass).reshape(M_ref.shape), 3 * M_ref) <= TOL_NORMWISE
    assert rel(host(ps.grid_mom).reshape(Q_ref.shape), 3 * Q_ref) <= TOL_NORMWISE


# ---------------------------------------------------------------- grid update + G2P

@pytest.mark.parametrize("bc_layers", [0, 1, 2])
def test_grid_update_parity(bc_layers):
    s = W.config0(2)
    pp, g, ps = particle_set(s, 8, dt=1e-3, bc_layers=bc_layers)
    ps.sort()
    ps.p2g()
    ps.grid_update()
    torch.cuda.synchronize()
    og = oracle_grid(g)
    M = host(ps.grid_mass).astype(np.float64).reshape(og.nz, og.ny, og.nx)
    Q = host(ps.grid_mom).astype(np.float64).reshape(3, og.nz, og.ny, og.nx)
    v_ref = O.grid_update(og, M, Q, 1e-3, s.gravity, bc_layers)
    v = host(ps.grid_vel).reshape(v_ref.shape)
    assert rel(v, v_ref) <= 1e-6
    assert np.array_equal(v[:, M == 0], np.zeros_like(v[:, M == 0]))


@pytest.mark.parametrize("n_modes", O.ALLOWED_N_MODES)
def test_g2p_parity(n_modes):
    """G2P from the device grid velocity (teacher-forced) against the oracle."""
    s = W.config0(3)
    note(f"g2p parity: config0 P={s.P} n_modes={n_modes}")
    pp, g, ps = particle_set(s, n_modes, dt=1e-3, bc_layers=1)
    ps.sort()
    ps.p2g()
    ps.grid_update()
    ps.g2p()
    torch.cuda.synchronize()
    og = oracle_grid(g)
    v = host(ps.grid_vel).astype(np.float64).reshape(3, og.nz, og.ny, og.nx)
    perm = host(ps.perm)
    xs = s.x[:, perm]
    c_ref, x_ref, _ = O.g2p(og, v, xs, n_modes, dt=1e-3)
    c = host(ps.coeff_next).reshape(3, n_modes, s.P)
    ec = rel(c, c_ref)
    per_mode = [rel(c[:, r], c_ref[:, r]) for r in range(n_modes)]
    note(f"  coeff {ec:.2e}  worst mode {max(per_mode):.2e}")
    assert ec <= TOL_NORMWISE
    norms = [np.linalg.norm(c_ref[:, r]) for r in range(n_modes)]
    for r in range(n_modes):
        if norms[r] >= 1e-3 * norms[0]:
            assert per_mode[r] <= TOL_NORMWISE, (r, per_mode[r])
    assert ulp_ok(host(ps.x_next), x_ref, 2, 1.0 + 4 / 32)


@pytest.mark.parametrize("n_modes", O.ALLOWED_N_MODES)
@pytest.mark.parametrize("variant", ["dt0_nowalls", "gravity_walls"])
@pytest.mark.parametrize("fused", [False, True])
def test_full_step_parity(n_modes, variant, fused):
    """Single-step parity case: sort -> P2G -> update -> G2P + advection on 32,768
    particles, against the oracle's own step (its own sort, P2G, update, G2P).  Fused, the
    G2P is polypic_g2p2g, after which the grid holds the P2G of the new state."""
    s = W.config0(0)
    dt, grav, bc = (0.0, (0.0, 0.0, 0.0), 0) if variant == "dt0_nowalls" else \
        (1e-4, (0.0, -9.8, 0.0), 1)
    note(f"step parity: config0 n_modes={n_modes} {variant} fused={fused}")
    pp, g, ps = particle_set(s, n_modes, dt=dt, gravity=grav, bc_layers=bc, fused=fused)
    ps.step()
    torch.cuda.synchronize()
    assert ps.status_flags() == 0
    ref = O.step(oracle_grid(g), s.x, s.coeff, n_modes, dt, grav, bc, sort=True)
    assert np.array_equal(host(ps.order), ref["perm"].astype(np.int64))
    if fused:
        check_grid_of_state(ps, oracle_grid(g), n_modes)
    else:
        assert rel(host(ps.grid_mass).reshape(ref["grid_mass"].shape),
                   ref["grid_mass"]) <= TOL_NORMWISE
        assert rel(host(ps.grid_mom).reshape(ref["grid_mom"].shape),
                   ref["grid_mom"]) <= TOL_NORMWISE
    c = host(ps.coeff).reshape(3, n_modes, s.P)
    assert rel(c, ref["coeff"]) <= TOL_NORMWISE
    assert ulp_ok(host(ps.x), ref["x"], 2, 1.0 + 4 / 32)


@pytest.mark.parametrize("fused", [False, True])
def test_f_and_mass_follow_the_permutation(fused):
    """Fabric-style set: per-point masses and deformation gradients (F' = (I + dt C) F)."""
    s = W.config2_fabric(0, n=64, side=120)
    note(f"fabric F update: P={s.P} fused={fused}")
    pp, g, ps = particle_set(s, 27, fused=fused)
    ps.step()
    torch.cuda.synchronize()
    assert ps.status_flags() == 0
    ref = O.step(oracle_grid(g), s.x, s.coeff, 27, s.dt, s.gravity, s.bc_layers, mass=s.mass,
                 F=s.F, sort=True)
    assert np.array_equal(host(ps.mass), s.mass[ref["perm"]])
    assert rel(host(ps.coeff).reshape(3, 27, s.P), ref["coeff"]) <= TOL_NORMWISE
    assert rel(host(ps.F), ref["F"]) <= 1e-6
    if fused:
        check_grid_of_state(ps, oracle_grid(g), 27, mass=ps.mass)
    else:
        assert rel(host(ps.grid_mass).reshape(ref["grid_mass"].shape),
                   ref["grid_mass"]) <= TOL_NORMWISE


# ---------------------------------------------------------------- G2P fused with the next P2G

@pytest.mark.parametrize("n_modes", O.ALLOWED_N_MODES)
def test_g2p2g_halves_against_the_oracle(n_modes):
    """One polypic_g2p2g call: its G2P half against the oracle's G2P of the same grid
    velocity (teacher-forced), its P2G half against the oracle's P2G of the state it wrote."""
    pp = require_gpu()
    s = W.config0(3)
    _, g, ps = particle_set(s, n_modes, dt=1e-3)
    og = oracle_grid(g)
    note(f"g2p2g: n_modes={n_modes} P={s.P}")
    ps.sort()
    ps.p2g()
    ps.grid_update()
    torch.cuda.synchronize()
    gv = host(ps.grid_vel).reshape(3, og.nz, og.ny, og.nx).astype(np.float64)
    src = host(ps.perm)
    ps.g2p2g()
    torch.cuda.synchronize()
    assert ps.status_flags() == 0
    c_ref, x_ref, _ = O.g2p(og, gv, s.x[:, src], n_modes, ps.dt)
    assert rel(host(ps.coeff_next).reshape(3, n_modes, s.P), c_ref) <= TOL_NORMWISE
    assert ulp_ok(host(ps.x_next), x_ref, 2, 1.0 + 4 / 32)
    M_ref, Q_ref = O.p2g(og, host(ps.x_next), host(ps.coeff_next).reshape(3, n_modes, s.P),
                         n_modes)
    assert rel(host(ps.grid_mass).reshape(M_ref.shape), M_ref) <= TOL_NORMWISE
    assert rel(host(ps.grid_mom).reshape(Q_ref.shape), Q_ref) <= TOL_NORMWISE


def test_g2p2g_with_mass_and_f_unsorted_ragged():
    """Per-particle mass and F, no permutation (input order), a ragged particle count."""
    pp = require_gpu()
    s = W.config2_fabric(1, n=64, side=97)        # 9,409 points: not a multiple of 256
    _, g, ps = particle_set(s, 27)
    og = oracle_grid(g)
    note(f"g2p2g with mass and F: P={s.P}")
    ps.p2g(use_perm=False)
    ps.grid_update()
    torch.cuda.synchronize()
    gv = host(ps.grid_vel).reshape(3, og.nz, og.ny, og.nx).astype(np.float64)
    ps.g2p2g(use_perm=False)
    torch.cuda.synchronize()
    assert ps.status_flags() == 0
    c_ref, x_ref, F_ref = O.g2p(og, gv, s.x, 27, ps.dt, s.F)
    assert rel(host(ps.coeff_next).reshape(3, 27, s.P), c_ref) <= TOL_NORMWISE
    assert rel(host(ps.F_next), F_ref) <= 1e-6
    assert np.array_equal(host(ps.mass_next), s.mass)
    M_ref, Q_ref = O.p2g(og, host(ps.x_next), host(ps.coeff_next).reshape(3, 27, s.P), 27,
                         s.mass)
    assert rel(host(ps.grid_mass).reshape(M_ref.shape), M_ref) <= TOL_NORMWISE
    assert rel(host(ps.grid_mom).reshape(Q_ref.shape), Q_ref) <= TOL_NORMWISE


def test_fused_steps_track_unfused_steps():
    """Eight steps of a moving scene, fused and unfused, from the same state: the same
    trajectory up to the order of the sums (and the permutations are identical)."""
    pp = require_gpu()
    s = W.config0(6)
    _, g, a = particle_set(s, 8, dt=2e-3, fused=True)
    _, _, b = particle_set(s, 8, dt=2e-3, fused=False)
    for k in range(8):
        a.step()
        b.step()
    torch.cuda.synchronize()
    assert a.status_flags() == 0 and b.status_flags() == 0

    def by_particle(ps, t):  # back to the original particle order
        out = torch.empty_like(t)
        out[..., ps.order] = t
        return host(out)
    assert rel(by_particle(a, a.x), by_particle(b, b.x)) <= 1e-6
    assert rel(by_particle(a, a.coeff), by_particle(b, b.coeff)) <= 1e-5


def test_g2p2g_empty_clears_the_grid():
    pp = require_gpu()
    g = pp.make_grid((12, 12, 12), 1 / 8)
    gm = torch.full((12 ** 3,), 7.0, device="cuda")
    gp = torch.full((3 * 12 ** 3,), 7.0, device="cuda")
    gv = torch.zeros(3 * 12 ** 3, device="cuda")
    e = torch.empty(0, device="cuda")
    pp.polypic_g2p2g(g, 27, 1e-4, gv, e, e.clone(), e.clone(), gm, gp)
    torch.cuda.synchronize()
    assert float(gm.abs().max()) == 0.0 and float(gp.abs().max()) == 0.0


def test_g2p2g_empty_accumulate_leaves_the_grid():
    pp = require_gpu()
    g = pp.make_grid((12, 12, 12), 1 / 8)
    gm = torch.full((12 ** 3,), 7.0, device="cuda")
    gp = torch.full((3 * 12 ** 3,), 5.0, device="cuda")
    gv = torch.zeros(3 * 12 ** 3, device="cuda")
    e = torch.empty(0, device="cuda")
    pp.polypic_g2p2g(g, 27, 1e-4, gv, e, e.clone(), e.clone(), gm, gp, accumulate=True)
    torch.cuda.synchronize()
    assert bool((gm == 7.0).all()) and bool((gp == 5.0).all())


def test_grid_update_clear_matches_grid_update_and_zeroes_its_inputs():
    """polypic_grid_update_clear: the same velocities bit for bit (same arithmetic per
    node), and the mass and momentum it read are left exactly zero."""
    pp = require_gpu()
    s = W.config0(4)
    _, g, ps = particle_set(s, 27, dt=1e-3, gravity=(0.0, -9.8, 0.0), bc_layers=1)
    ps.sort()
    ps.p2g()
    ps.grid_update()
    torch.cuda.synchronize()
    v_ref = host(ps.grid_vel).copy()
    assert float(ps.grid_mass.max()) > 0.0
    ps.grid_vel.fill_(123.0)
    ps.grid_update(clear=True)
    torch.cuda.synchronize()
    assert np.array_equal(host(ps.grid_vel), v_ref)
    assert float(ps.grid_mass.abs().max()) == 0.0 and float(ps.grid_mom.abs().max()) == 0.0
    assert not ps.grid_current


@pytest.mark.parametrize("n_modes", [4, 27])
def test_g2p2g_accumulates_into_a_given_grid(n_modes):
    """polypic_g2p2g with accumulate = 1 onto a grid that already holds sums: the result
    is those sums plus the oracle's P2G of the state the call wrote."""
    pp = require_gpu()
    s = W.config0(5)
    _, g, ps = particle_set(s, n_modes, dt=1e-3)
    og = oracle_grid(g)
    note(f"g2p2g accumulate: n_modes={n_modes} P={s.P}")
    ps.sort()
    ps.p2g()
    ps.grid_update()
    rng = np.random.default_rng(11)
    M0 = rng.random(og.n_nodes).astype(np.float32)
    Q0 = rng.standard_normal(3 * og.n_nodes).astype(np.float32)
    ps.grid_mass.copy_(torch.from_numpy(M0))
    ps.grid_mom.copy_(torch.from_numpy(Q0))
    ps.g2p2g(accumulate=True)
    torch.cuda.synchronize()
    assert ps.status_flags() == 0
    M_ref, Q_ref = O.p2g(og, host(ps.x_next), host(ps.coeff_next).reshape(3, n_modes, s.P),
                         n_modes)
    M_ref = M_ref + M0.astype(np.float64).reshape(M_ref.shape)
    Q_ref = Q_ref + Q0.astype(np.float64).reshape(Q_ref.shape)
    assert rel(host(ps.grid_mass).reshape(M_ref.shape), M_ref) <= TOL_NORMWISE
    assert rel(host(ps.grid_mom).reshape(Q_ref.shape), Q_ref) <= TOL_NORMWISE


# ---------------------------------------------------------------- exact fixture and edges

@pytest.mark.parametrize("case_idx", range(4))
def test_exact_golden_fixture(case_idx):
    """Six hand-placed particles (t = -1/2, 0, 1/2 - 2^-20) against exact rationals."""
    pp = require_gpu()
    with open(GOLDEN) as f:
        doc = json.load(f)
    case = doc["cases"][case_idx]
    n_modes = case["n_modes"]
    fr = lambda v: float(Fr(v))  # noqa: E731
    g = pp.make_grid(doc["nodes"], fr(doc["dx"]), [fr(o) for o in doc["origin"]],
                     fr(doc["inv_dx"]))
    x = np.array([[fr(v) for v in p] for p in doc["x"]], np.float32).T.copy()
    mass = np.array([fr(m) for m in doc["mass"]], np.float32)
    cin = np.array([[[fr(v) for v in ca] for ca in c] for c in doc["coeff_in"]])
    cin = np.ascontiguousarray(np.transpose(cin, (1, 2, 0))[:, :n_modes]).astype(np.float32)
    ps = pp.ParticleSet(g, n_modes, dev(x), dev(cin), mass=dev(mass), dt=fr(doc["dt"]),
                        gravity=[fr(v) for v in doc["gravity"]], bc_layers=doc["bc_layers"])
    ps.p2g(use_perm=False)
    ps.grid_update()
    ps.g2p(use_perm=False)
    torch.cuda.synchronize()
    nx, ny, nz = doc["nodes"]
    M = host(ps.grid_mass).reshape(nz, ny, nx)
    Q = host(ps.grid_mom).reshape(3, nz, ny, nx)
    m_ref = np.zeros_like(M, dtype=np.float64)
    q_ref = np.zeros_like(Q, dtype=np.float64)
    for nd, ms, psx in zip(case["nodes"], case["grid_mass"], case["grid_mom"]):
        m_ref[nd[2], nd[1], nd[0]] = fr(ms)
        q_ref[:, nd[2], nd[1], nd[0]] = [fr(v) for v in psx]
    assert rel(M, m_ref) <= TOL_NORMWISE and rel(Q, q_ref) <= TOL_NORMWISE
    c_ref = np.array([[[fr(v) for v in ca] for ca in cp] for cp in case["coeff"]])
    c = np.transpose(host(ps.coeff_next).reshape(3, n_modes, -1), (2, 0, 1))
    assert rel(c, c_ref) <= TOL_NORMWISE
    assert ulp_ok(host(ps.x_next), np.array(case["x_out"], np.float32).T, 2, 2.0)


def test_empty_and_single_particle():
    pp = require_gpu()
    g = pp.make_grid((12, 12, 12), 1 / 8)
    gm = torch.full((12 ** 3,), 7.0, device="cuda")
    gp = torch.full((3 * 12 ** 3,), 7.0, device="cuda")
    x0 = torch.empty(0, device="cuda")
    c0 = torch.empty(0, device="cuda")
    pp.polypic_p2g(g, 27, x0, c0, gm, gp)          # P = 0: only the clear
    torch.cuda.synchronize()
    assert float(gm.abs().max()) == 0.0 and float(gp.abs().max()) == 0.0
    x = np.array([[0.61], [0.7], [0.83]], np.float32)
    c = np.random.default_rng(0).standard_normal((3, 27, 1)).astype(np.float32)
    ps = pp.ParticleSet(g, 27, dev(x), dev(c), dt=0.0, gravity=(0, 0, 0), bc_layers=0)
    ps.step()
    torch.cuda.synchronize()
    # one particle alone: the 27-mode round trip returns its own coefficients
    assert rel(host(ps.coeff).reshape(3, 27, 1), c) <= 1e-5


def test_degenerate_offsets_t_minus_half():
    """Particles exactly on u = k + 1/2 (t = -1/2 on one or more axes)."""
    pp = require_gpu()
    n = 16
    g = pp.make_grid((n + 4,) * 3, 1 / n)
    rng = np.random.default_rng(1)
    P = 4096
    u = rng.integers(4, n, size=(3, P)) + rng.integers(0, 8, size=(3, P)) / 8.0
    u[:, : P // 2] = np.floor(u[:, : P // 2]) + 0.5      # t = -1/2 on all axes
    u[0, P // 2:] = np.floor(u[0, P // 2:]) + 0.5        # t = -1/2 on x only
    x = (u / n).astype(np.float32)
    c = (rng.standard_normal((3, 27, P)) * 0.3).astype(np.float32)
    ps = pp.ParticleSet(g, 27, dev(x), dev(c), dt=1e-4, bc_layers=1, fused=False)
    ps.step()
    torch.cuda.synchronize()
    og = oracle_grid(g)
    ref = O.step(og, x, c, 27, 1e-4, (0.0, -9.8, 0.0), 1, sort=True)
    assert rel(host(ps.grid_mom).reshape(ref["grid_mom"].shape), ref["grid_mom"]) <= TOL_NORMWISE
    assert rel(host(ps.coeff).reshape(3, 27, P), ref["coeff"]) <= TOL_NORMWISE


def test_out_of_range_particle_is_flagged_and_skipped():
    pp = require_gpu()
    g = pp.make_grid((12, 12, 12), 1 / 8)
    x = np.array([[0.6, 0.01, 0.7], [0.6, 0.6, 0.7], [0.6, 0.6, 5.0]], np.float32)
    c = np.ones((3, 4, 3), np.float32)
    ps = pp.ParticleSet(g, 4, dev(x), dev(c), dt=0.0, gravity=(0, 0, 0), bc_layers=0)
    ps.p2g(use_perm=False)
    torch.cuda.synchronize()
    assert ps.status_flags() & 1
    assert abs(float(ps.grid_mass.sum()) - 1.0) < 1e-6   # only the in-range particle
    ps.status.zero_()
    ps.sort()
    torch.cuda.synchronize()
    assert ps.status_flags() & 1
    assert sorted(host(ps.perm).tolist()) == [0, 1, 2]


def test_invalid_permutation_never_faults():
    """A caller permutation with out-of-range entries is clamped (wrong data, no fault)."""
    pp = require_gpu()
    s = W.random_scene(8, 16, 1000)
    g = pp.grid_from_spec(s.grid)
    ps = pp.ParticleSet(g, 4, dev(s.x), dev(s.coeff[:, :4]))
    bad = torch.full((s.P,), 1 << 30, dtype=torch.int32, device="cuda")
    bad[::2] = -7
    pp.polypic_p2g(g, 4, ps.x, ps.coeff, ps.grid_mass, ps.grid_mom, perm=bad)
    pp.polypic_g2p(g, 4, 1e-4, ps.grid_vel.zero_(), ps.x, ps.coeff_next, perm=bad)
    torch.cuda.synchronize()
    assert torch.isfinite(ps.grid_mass).all()


def test_stale_keys_are_flagged_not_trusted():
    """Cell path: keys that no longer match the positions: those particles are skipped and
    flagged (the brick path recomputes every stencil from the positions)."""
    pp = require_gpu()
    s = W.config0(5)
    pp_, g, ps = particle_set(s, 8)
    ps.sort()
    moved = ps.perm[:100].long()
    ps.x[0, moved] += 1.5 / 32   # moves 100 particles by 1.5 cells along x
    with p2g_config(pp, 8, pp.POLYPIC_P2G_CELLS, 512):
        ps.p2g()
        torch.cuda.synchronize()
    assert ps.status_flags() & 1
    total = float(ps.grid_mass.double().sum())
    assert abs(total - (s.P - 100)) < 1e-3


def test_cell_path_with_sparse_and_dense_cells():
    """Cells holding 1 .. 40 particles, tiles split across the sorted array."""
    pp = require_gpu()
    rng = np.random.default_rng(12)
    n = 24
    counts = rng.integers(0, 41, size=200)
    cells = rng.integers(3, n - 3, size=(200, 3))
    xs = []
    for cnt, cc in zip(counts, cells):
        xs.append((cc[:, None] + 2 + rng.random((3, cnt))) / n)
    x = np.concatenate(xs, axis=1).astype(np.float32)
    P = x.shape[1]
    c = (rng.standard_normal((3, 27, P)) * 0.3).astype(np.float32)
    mass = (0.5 + rng.random(P)).astype(np.float32)
    g = pp.make_grid((n + 4,) * 3, 1 / n)
    ps = pp.ParticleSet(g, 27, dev(x), dev(c), mass=dev(mass))
    ps.sort()
    M_ref, Q_ref = O.p2g(oracle_grid(g), x, c, 27, mass)
    for path in (pp.POLYPIC_P2G_CELLS, pp.POLYPIC_P2G_BRICKS):
        with p2g_config(pp, 27, path, 512 if path == pp.POLYPIC_P2G_CELLS else 256):
            ps.p2g()
            torch.cuda.synchronize()
        assert rel(host(ps.grid_mass).reshape(M_ref.shape), M_ref) <= TOL_NORMWISE, path
        assert rel(host(ps.grid_mom).reshape(Q_ref.shape), Q_ref) <= TOL_NORMWISE, path
    assert ps.status_flags() == 0


@pytest.mark.parametrize("n_modes", [4, 27])
def test_every_p2g_configuration_and_the_autotuner(n_modes):
    """Each P2G launch configuration (cell runs; FP64 bricks of 2^3, 4^3 or 8^3 cells with
    256 or 512 threads, in index order, XCD order or persistent) matches the oracle, in sort
    order and in input order (runs beyond the bricks go to HBM); the autotuner returns one of
    them and leaves a valid result."""
    pp = require_gpu()
    s = W.config0(4)
    pp_, g, ps = particle_set(s, n_modes)
    ps.sort()
    M_ref, Q_ref = O.p2g(oracle_grid(g), s.x, s.coeff, n_modes)
    try:
        configs = [(1, 512, 0, 0, 4)] + [(0, b, sc, pc, e) for e in (4, 2, 8) for b in (256, 512)
                                         for sc, pc in ((0, 0), (1, 0), (2, 1), (2, 4))]
        for cfg in configs:
            pp.polypic_set_p2g_config(n_modes, *cfg)
            for use_perm in ((True, False) if cfg[0] == 0 else (True,)):
                ps.p2g(use_perm=use_perm)
                torch.cuda.synchronize()
                M = host(ps.grid_mass).reshape(M_ref.shape)
                Q = host(ps.grid_mom).reshape(Q_ref.shape)
                assert rel(M, M_ref) <= TOL_NORMWISE, (cfg, use_perm)
                assert rel(Q, Q_ref) <= TOL_NORMWISE, (cfg, use_perm)
        choice = ps.autotune()
        assert (choice.path, choice.block) in [(1, 512), (0, 256), (0, 512)]
        assert choice.schedule in (pp.POLYPIC_SCHED_LINEAR, pp.POLYPIC_SCHED_XCD)
        assert choice.brick in (2, 4, 8)
        assert pp.polypic_get_p2g_config(n_modes) == choice
        assert rel(host(ps.grid_mom).reshape(Q_ref.shape), Q_ref) <= TOL_NORMWISE
    finally:
        pp.polypic_set_p2g_config(n_modes, -1, 256)


@pytest.mark.parametrize("n_modes", [4, 27])
def test_p2g_lane_groups_with_every_cell_size(n_modes):
    """Cells holding 1 .. 9 particles in turn (so that in sorted order the runs of one cell
    start at every offset of the lane pairs and quads that pre-add their nodal values), with
    out-of-range particles among them: every particle is counted exactly once."""
    pp = require_gpu()
    rng = np.random.default_rng(11)
    gs = W.cubic_grid(32)
    cells = [(cx, cy, cz) for cz in range(4, 28, 2) for cy in range(4, 28, 3) for cx in range(4, 28)]
    xs = []
    for k, (cx, cy, cz) in enumerate(cells):
        n = 1 + k % 9
        u = rng.random((3, n))
        xs.append(np.stack([(2 + cx + u[0]) * gs.dx, (2 + cy + u[1]) * gs.dx,
                            (2 + cz + u[2]) * gs.dx]))
    x = np.concatenate(xs, axis=1).astype(np.float32)
    P = x.shape[1]
    bad = rng.choice(P, size=37, replace=False)
    x[0, bad] = -1.0                                  # outside the grid: skipped and flagged
    c = np.zeros((3, 27, P), np.float32)
    c[:, 0] = rng.standard_normal((3, P))
    c[:, 1:] = 0.1 * rng.standard_normal((3, 26, P))
    m = (0.5 + rng.random(P)).astype(np.float32)
    note(f"p2g lane groups: P={P} n_modes={n_modes}")
    g = pp.grid_from_spec(gs)
    ps = pp.ParticleSet(g, n_modes, dev(x), dev(c[:, :n_modes]), mass=dev(m))
    good = np.setdiff1d(np.arange(P), bad)
    M_ref, Q_ref = O.p2g(oracle_grid(g), x[:, good], c[:, :, good], n_modes, m[good])
    ps.sort()
    configs = [(0, 256, 0, 0, 4), (0, 512, 0, 0, 4), (0, 256, 1, 0, 4), (0, 256, 2, 2, 4),
               (1, 512, 0, 0, 4), (0, 256, 0, 0, 2), (0, 512, 1, 0, 2), (0, 256, 0, 0, 8),
               (0, 512, 2, 2, 8)]
    try:
        for cfg in configs:
            pp.polypic_set_p2g_config(n_modes, *cfg)
            ps.status.zero_()
            ps.p2g()
            torch.cuda.synchronize()
            assert ps.status_flags() & 1
            assert rel(host(ps.grid_mass).reshape(M_ref.shape), M_ref) <= TOL_NORMWISE, cfg
            assert rel(host(ps.grid_mom).reshape(Q_ref.shape), Q_ref) <= TOL_NORMWISE, cfg
    finally:
        pp.polypic_set_p2g_config(n_modes, -1, 256)


# ---------------------------------------------------------------- incremental re-sort

def _resort(pp, g, x, keys_prev, P):
    keys = torch.zeros(P, dtype=torch.int32, device="cuda")
    perm = torch.zeros(P, dtype=torch.int32, device="cuda")
    ws = torch.empty(pp.ops.polypic_sort_update_workspace_bytes(g, P), dtype=torch.uint8,
                     device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    pp.ops.polypic_sort_update(g, x, keys_prev, keys, perm, ws, status)
    torch.cuda.synchronize()
    return keys, perm, int(status.item())


def _full_sort(pp, g, x, P):
    keys = torch.empty(P, dtype=torch.int32, device="cuda")
    perm = torch.empty(P, dtype=torch.int32, device="cuda")
    ws = torch.empty(pp.ops.polypic_sort_workspace_bytes(g, P), dtype=torch.uint8, device="cuda")
    pp.ops.polypic_sort(g, x, keys, perm, ws)
    torch.cuda.synchronize()
    return keys, perm


def test_resort_over_steps_equals_full_sort_and_oracle():
    """Ten steps of a moving set: every step's incremental re-sort gives exactly the full
    sort's and the oracle's stable argsort."""
    pp = require_gpu()
    s = W.config0(6)
    pp_, g, ps = particle_set(s, 8, dt=2e-3)          # larger dt: more cell changes per step
    og = oracle_grid(g)
    changed_total = 0
    for k in range(10):
        x_before = host(ps.x).copy()
        ps.sort()
        torch.cuda.synchronize()
        keys_ref, perm_ref = O.sort_keys(og, x_before)
        assert np.array_equal(host(ps.keys).view(np.uint32), keys_ref), k
        assert np.array_equal(host(ps.perm), perm_ref), k
        if k > 0:
            changed_total += int((host(ps.slot_keys).view(np.uint32) !=
                                  O.morton_key(O.stencil_base(og, x_before)[0])).sum())
        ps.p2g()
        ps.grid_update()
        ps.g2p()
        ps.swap()
    assert changed_total > 0                 # the incremental path did reorder something
    assert ps.status_flags() == 0


def test_resort_after_a_sort_without_a_step_keeps_its_reference():
    """A sort that no step follows (the autotuner's) leaves the particle arrays in place, so
    the next re-sort still starts from the keys the slot order was sorted under: few slots
    count as changed, and the result is still the exact stable sort."""
    pp = require_gpu()
    s = W.config0(7)
    _, g, ps = particle_set(s, 8, dt=2e-3)
    og = oracle_grid(g)
    for _ in range(2):
        ps.step()
    ps.sort()                                        # no step after this one
    for k in range(2):
        x_before = host(ps.x).copy()
        ps.sort()
        torch.cuda.synchronize()
        keys_ref, perm_ref = O.sort_keys(og, x_before)
        assert np.array_equal(host(ps.keys).view(np.uint32), keys_ref), k
        assert np.array_equal(host(ps.perm), perm_ref), k
        slot_ref = O.morton_key(O.stencil_base(og, x_before)[0])
        changed = float((host(ps.slot_keys).view(np.uint32) != slot_ref).mean())
        note(f"  step {k}: fraction of slots changed {changed:.4f}")
        assert changed < 0.1, changed
        ps.p2g()
        ps.grid_update()
        ps.g2p()
        ps.swap()
    assert ps.status_flags() == 0


@pytest.mark.parametrize("case", ["half", "all", "none", "out_of_range"])
def test_resort_cases(case):
    pp = require_gpu()
    s = W.random_scene(9, 32, 50000)
    g = pp.grid_from_spec(s.grid)
    og = oracle_grid(g)
    P = s.P
    x0 = dev(s.x)
    keys0, perm0 = _full_sort(pp, g, x0, P)
    xs = x0[:, perm0.long()].contiguous()            # the particle arrays in sort order
    rng = np.random.default_rng(3)
    xh = host(xs).copy()
    if case == "half":
        pick = rng.random(P) < 0.5
        xh[:, pick] += (rng.integers(-2, 3, size=(3, int(pick.sum()))) / 32.0).astype(np.float32)
        xh = np.clip(xh, 2.5 / 32, 1 + 1.5 / 32).astype(np.float32)
    elif case == "all":
        xh[0] += np.float32(1.0 / 32)
    elif case == "out_of_range":
        pick = rng.choice(P, size=50, replace=False)
        xh[1, pick] = -3.0
    xn = dev(xh)
    note(f"resort case {case}: P={P}")
    keys, perm, status = _resort(pp, g, xn, keys0, P)
    keys_f, perm_f = _full_sort(pp, g, xn, P)
    assert torch.equal(keys, keys_f) and torch.equal(perm, perm_f)
    if case != "out_of_range":
        keys_ref, perm_ref = O.sort_keys(og, xh)
        assert np.array_equal(host(perm), perm_ref)
        assert status == 0
    else:
        assert status & 1


def test_resort_many_changed_across_many_workgroups():
    """A re-sort whose changed list spans many sort tiles and whose compaction runs in far
    more workgroups than there are copies of the digit totals (each workgroup adds into
    copy b mod 32): half of the particles in the lower half of the domain move one cell up."""
    pp = require_gpu()
    s = W.random_scene(12, 48, 400000)
    g = pp.grid_from_spec(s.grid)
    og = oracle_grid(g)
    P = s.P
    x0 = dev(s.x)
    keys0, perm0 = _full_sort(pp, g, x0, P)
    xh = host(x0[:, perm0.long()].contiguous()).copy()
    rng = np.random.default_rng(5)
    pick = (xh[2] < 0.5) & (rng.random(P) < 0.5)
    xh[2, pick] += np.float32(1.0 / 48)
    note(f"resort many changed: P={P}, moved {int(pick.sum())}")
    keys, perm, status = _resort(pp, g, dev(xh), keys0, P)
    keys_ref, perm_ref = O.sort_keys(og, xh)
    assert status == 0
    assert np.array_equal(host(keys).view(np.uint32), keys_ref)
    assert np.array_equal(host(perm), perm_ref)


def test_resort_changed_list_longer_than_the_scatter_grid():
    """Every particle changes cell and the changed list has more sort tiles (600) than the
    scatter launches workgroups (512), so workgroups claim a second tile."""
    pp = require_gpu()
    P = 600 * 2048 - 77                              # ragged last tile
    s = W.random_scene(13, 64, P)
    g = pp.grid_from_spec(s.grid)
    og = oracle_grid(g)
    x0 = dev(s.x)
    keys0, perm0 = _full_sort(pp, g, x0, P)
    xh = host(x0[:, perm0.long()].contiguous()).copy()
    xh[0] += np.float32(1.0 / 64)
    note(f"resort all changed, long list: P={P}")
    keys, perm, status = _resort(pp, g, dev(xh), keys0, P)
    keys_ref, perm_ref = O.sort_keys(og, xh)
    assert status == 0
    assert np.array_equal(host(keys).view(np.uint32), keys_ref)
    assert np.array_equal(host(perm), perm_ref)


def test_resort_with_more_workgroups_than_the_folded_scan_takes():
    """More than 4096 slot tiles of 2048 (8.39 M particles): the re-sort scans the
    per-workgroup counts in a launch of its own instead of summing them in every
    workgroup of the compaction.  Half of the particles in the lower half move a cell."""
    pp = require_gpu()
    P = 4097 * 2048 + 5
    n = 96
    spec = W.cubic_grid(n)
    g = pp.grid_from_spec(spec)
    og = oracle_grid(g)
    rng = np.random.default_rng(14)
    x = (4.0 / n + rng.random((3, P)) * ((n - 4.0) / n)).astype(np.float32)
    x0 = dev(x)
    keys0, perm0 = _full_sort(pp, g, x0, P)
    xh = host(x0[:, perm0.long()].contiguous()).copy()
    del x0
    pick = (xh[2] < 0.5) & (rng.random(P) < 0.5)
    xh[2, pick] += np.float32(1.0 / n)
    note(f"resort beyond the folded scan: P={P}, moved {int(pick.sum())}")
    keys, perm, status = _resort(pp, g, dev(xh), keys0, P)
    keys_ref, perm_ref = O.sort_keys(og, xh)
    assert status == 0
    assert np.array_equal(host(keys).view(np.uint32), keys_ref)
    assert np.array_equal(host(perm), perm_ref)


def test_resort_with_unordered_previous_keys_is_flagged_and_in_range():
    pp = require_gpu()
    s = W.random_scene(10, 24, 20000)
    g = pp.grid_from_spec(s.grid)
    P = s.P
    x = dev(s.x)
    bogus = torch.randint(0, 1 << 20, (P,), dtype=torch.int32, device="cuda")  # not ascending
    keys, perm, status = _resort(pp, g, x, bogus, P)
    assert status & 2
    p = host(perm)
    assert p.min() >= 0 and p.max() < P


@pytest.mark.parametrize("order", ["linear", "xcd"])
@pytest.mark.parametrize("n_modes", [4, 27])
@pytest.mark.parametrize("case", ["parity_8ppc", "fluid_16ppc", "fabric_mass_f_ragged"])
def test_g2p2g_lane_quads_against_the_oracle(n_modes, case, order):
    """polypic_g2p2g with lane groups of 4, chunks in launch or XCD order (set explicitly,
    then restored): both halves against the oracle as for pairs, at 8 and 16 particles per
    cell and with per-point mass and F in input order (a ragged count), so that quads that
    straddle cells fall back to pairs or single lanes."""
    pp = require_gpu()
    sched = pp._lib.POLYPIC_SCHED_XCD if order == "xcd" else pp._lib.POLYPIC_SCHED_LINEAR
    if case == "parity_8ppc":
        s = W.config0(3)
    elif case == "fluid_16ppc":
        s = W.config2_fluid(2, n=32)
    else:
        s = W.config2_fabric(1, n=64, side=97)
    sort = case != "fabric_mass_f_ragged"
    _, g, ps = particle_set(s, n_modes, dt=1e-3)
    og = oracle_grid(g)
    note(f"g2p2g quads: {case} n_modes={n_modes} P={s.P}")
    pp.ops.polypic_set_g2p2g_config(n_modes, 4, sched)
    try:
        assert tuple(pp.ops.polypic_get_g2p2g_config(n_modes)) == (4, sched)
        if sort:
            ps.sort()
        ps.p2g(use_perm=sort)
        ps.grid_update()
        torch.cuda.synchronize()
        gv = host(ps.grid_vel).reshape(3, og.nz, og.ny, og.nx).astype(np.float64)
        src = host(ps.perm) if sort else np.arange(s.P)
        ps.g2p2g(use_perm=sort)
        torch.cuda.synchronize()
    finally:
        pp.ops.polypic_set_g2p2g_config(n_modes, -1, -1)
    assert tuple(pp.ops.polypic_get_g2p2g_config(n_modes)) == (2, pp._lib.POLYPIC_SCHED_LINEAR)
    assert ps.status_flags() == 0
    F_in = None if s.F is None else s.F[:, src]
    c_ref, x_ref, F_ref = O.g2p(og, gv, s.x[:, src], n_modes, ps.dt, F_in)
    assert rel(host(ps.coeff_next).reshape(3, n_modes, s.P), c_ref) <= TOL_NORMWISE
    m_new = None if s.mass is None else host(ps.mass_next)
    M_ref, Q_ref = O.p2g(og, host(ps.x_next), host(ps.coeff_next).reshape(3, n_modes, s.P),
                         n_modes, m_new)
    assert rel(host(ps.grid_mass).reshape(M_ref.shape), M_ref) <= TOL_NORMWISE
    assert rel(host(ps.grid_mom).reshape(Q_ref.shape), Q_ref) <= TOL_NORMWISE


def test_g2p2g_autotuner_picks_a_lane_group_and_keeps_results():
    """ParticleSet.autotune_fused: the library times pairs and quads, in launch and in XCD
    chunk order, on the set's data, keeps one, and the step it ran is a correct fused step
    (its P2G half against the oracle)."""
    pp = require_gpu()
    s = W.config2_fluid(4, n=32)
    _, g, ps = particle_set(s, 27, dt=1e-3)
    og = oracle_grid(g)
    try:
        choice = ps.autotune_fused()
        assert choice.lane_group in (2, 4)
        assert choice.schedule in (pp._lib.POLYPIC_SCHED_LINEAR, pp._lib.POLYPIC_SCHED_XCD)
        assert pp.ops.polypic_get_g2p2g_config(27) == choice
        torch.cuda.synchronize()
        assert ps.status_flags() == 0 and ps.grid_current
        M_ref, Q_ref = O.p2g(og, host(ps.x), host(ps.coeff).reshape(3, 27, s.P), 27)
        assert rel(host(ps.grid_mass).reshape(M_ref.shape), M_ref) <= TOL_NORMWISE
        assert rel(host(ps.grid_mom).reshape(Q_ref.shape), Q_ref) <= TOL_NORMWISE
    finally:
        pp.ops.polypic_set_g2p2g_config(27, -1, -1)
