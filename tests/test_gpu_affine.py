"""P2G with the affine back-map of Eq. 12 on the GPU (polypic_p2g_affine) against the FP64
oracle's p2g_affine: modes at (I + dt C)^-1 (x_i - x_p) / dx with the quadratic factor
of the fitting position.  Bar: normwise 1e-5 on grid mass and momentum."""
import json
import os
from fractions import Fraction as Fr

import numpy as np
import pytest
import torch

import workloads as W
from oracle import polypic_oracle as O
from tests.gpu_util import (TOL_NORMWISE, dev, host, note, oracle_grid, particles_touching, rel,
                            require_gpu, sample_nodes)

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tiny_exact_affine.json")


def _scene(seed, n=24, P=20_001):
    rng = np.random.default_rng(seed)
    g = W.cubic_grid(n)
    u = 3.0 + rng.random((3, P)) * (n - 2.0)
    x = (u / n).astype(np.float32)
    x_fit = (x - (0.3 * rng.standard_normal((3, P))) / n).astype(np.float32)
    c = np.zeros((3, 27, P), np.float32)
    c[:, 0] = rng.standard_normal((3, P))
    c[:, 1:] = 0.3 * rng.standard_normal((3, 26, P))
    m = (0.5 + rng.random(P)).astype(np.float32)
    return g, x, x_fit, c, m


def _device_p2g(pp, g, nm, dt, x, c, x_fit=None, m=None, sort=True):
    P = x.shape[1]
    N = pp.ops.n_nodes(g)
    xd = dev(x)
    perm = None
    if sort:
        keys = torch.empty(P, dtype=torch.int32, device="cuda")
        perm = torch.empty(P, dtype=torch.int32, device="cuda")
        ws = torch.empty(pp.ops.polypic_sort_workspace_bytes(g, P), dtype=torch.uint8,
                         device="cuda")
        pp.ops.polypic_sort(g, xd, keys, perm, ws)
    gm = torch.empty(N, device="cuda")
    gp = torch.empty(3 * N, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    pp.ops.polypic_p2g_affine(g, nm, dt, xd, dev(c[:, :nm]), gm, gp,
                              x_fit=None if x_fit is None else dev(x_fit),
                              mass=None if m is None else dev(m), perm=perm, status_dev=st)
    torch.cuda.synchronize()
    return host(gm).astype(np.float64), host(gp).astype(np.float64), int(st.item())


@pytest.mark.parametrize("n_modes", [1, 4, 8, 27])
@pytest.mark.parametrize("sort", [True, False])
def test_affine_p2g_matches_oracle(n_modes, sort):
    pp = require_gpu()
    gs, x, x_fit, c, m = _scene(1)
    g = pp.grid_from_spec(gs)
    og = oracle_grid(g)
    dt = 2e-3
    note(f"affine p2g: n_modes={n_modes} sort={sort}")
    gm, gp, st = _device_p2g(pp, g, n_modes, dt, x, c, x_fit, m, sort)
    assert st == 0
    M, Q = O.p2g_affine(og, x, c, n_modes, dt, x_fit=x_fit, mass=m)
    e_m, e_p = rel(gm, M.ravel()), rel(gp, Q.ravel())
    note(f"  mass {e_m:.2e} momentum {e_p:.2e}")
    assert e_m <= TOL_NORMWISE and e_p <= TOL_NORMWISE


def test_affine_p2g_at_zero_dt_equals_polypic_p2g():
    """dt = 0 without x_fit is the plain P2G (Eq. 13).  The two kernels sum in different
    float32 orders (mode products per node against three separable contractions), so
    they agree to the parity bar, not bit for bit."""
    pp = require_gpu()
    gs, x, _, c, m = _scene(2)
    g = pp.grid_from_spec(gs)
    gm, gp, _ = _device_p2g(pp, g, 27, 0.0, x, c, None, m)
    N = pp.ops.n_nodes(g)
    gm0 = torch.empty(N, device="cuda")
    gp0 = torch.empty(3 * N, device="cuda")
    pp.ops.polypic_p2g(g, 27, dev(x), dev(c), gm0, gp0, mass=dev(m))
    torch.cuda.synchronize()
    assert rel(gm, host(gm0)) <= TOL_NORMWISE and rel(gp, host(gp0)) <= TOL_NORMWISE


@pytest.mark.parametrize("case_idx", range(4))
def test_affine_p2g_exact_golden_fixture(case_idx):
    pp = require_gpu()
    with open(GOLDEN) as f:
        doc = json.load(f)
    case = doc["cases"][case_idx]
    nm = case["n_modes"]
    g = pp.make_grid(doc["nodes"], float(Fr(doc["dx"])))
    og = oracle_grid(g)
    x = np.array([[float(Fr(v)) for v in p] for p in doc["x"]], np.float32).T
    xf = np.array([[float(Fr(v)) for v in p] for p in doc["x_fit"]], np.float32).T
    mass = np.array([float(Fr(v)) for v in doc["mass"]], np.float32)
    cin = np.array([[[float(Fr(v)) for v in ca] for ca in c] for c in doc["coeff_in"]])
    cin = np.ascontiguousarray(np.transpose(cin, (1, 2, 0)).astype(np.float32))
    gm, gp, st = _device_p2g(pp, g, nm, float(Fr(doc["dt"])), x, cin, xf, mass, sort=False)
    assert st == 0
    Me = np.zeros((og.nz, og.ny, og.nx))
    Qe = np.zeros((3, og.nz, og.ny, og.nx))
    for nd, ms, ps in zip(case["nodes"], case["grid_mass"], case["grid_mom"]):
        ix, iy, iz = nd
        Me[iz, iy, ix] = float(Fr(ms))
        for a in range(3):
            Qe[a, iz, iy, ix] = float(Fr(ps[a]))
    assert rel(gm, Me.ravel()) <= TOL_NORMWISE
    assert rel(gp, Qe.ravel()) <= TOL_NORMWISE


def test_affine_singular_map_is_flagged_and_skipped():
    """I + dt C singular (C_xx = -1/dt, exact in float32): the particle is flagged and
    contributes nothing."""
    pp = require_gpu()
    g = pp.make_grid((12, 12, 12), 1 / 8)
    x = np.array([[0.6, 0.7], [0.6, 0.6], [0.6, 0.65]], np.float32)
    c = np.zeros((3, 4, 2), np.float32)
    dt = 0.125
    c[0, 1, 0] = -1.0                 # dt * coeff[0][1] / dx = -1: A_xx = 0
    gm, _, st = _device_p2g(pp, g, 4, dt, x, c, sort=False)
    assert st & pp._lib.POLYPIC_FLAG_MAP
    assert abs(gm.sum() - 1.0) < 1e-6


def test_affine_steps_teacher_forced():
    """Three steps of the affine-map set on the 32^3-cell parity case with dt = 1e-3 (each
    step's P2G carries the coefficients fitted at the previous positions), then the fourth
    step's P2G against the oracle on the device state."""
    pp = require_gpu()
    s = W.config0(0)
    g = pp.grid_from_spec(s.grid)
    og = oracle_grid(g)
    ps = pp.AffineParticleSet(g, 27, dev(s.x), dev(s.coeff), dt=1e-3, gravity=s.gravity,
                              bc_layers=1)
    for _ in range(3):
        ps.step()
    torch.cuda.synchronize()
    assert ps.fit_valid
    x, xf = host(ps.x).copy(), host(ps.x_fit).copy()
    c = host(ps.coeff).reshape(3, 27, ps.P).copy()
    assert np.abs(x - xf).max() > 0          # the particles moved since the fit
    ps.sort()
    ps.p2g()
    torch.cuda.synchronize()
    assert ps.status_flags() == 0
    M, Q = O.p2g_affine(og, x, c, 27, ps.dt, x_fit=xf)
    e_m = rel(host(ps.grid_mass), M.ravel())
    e_p = rel(host(ps.grid_mom), Q.ravel())
    note(f"affine steps: mass {e_m:.2e} momentum {e_p:.2e}")
    assert e_m <= TOL_NORMWISE and e_p <= TOL_NORMWISE


def test_affine_full_size_sampled():
    """The moving dam break (4,194,304 particles, 27 modes) stepped twice with the affine
    map; the next P2G at sampled nodes against the oracle over the particles touching them."""
    pp = require_gpu()
    s = W.config1_moving(0)
    g = pp.grid_from_spec(s.grid)
    og = oracle_grid(g)
    ps = pp.AffineParticleSet(g, 27, dev(s.x), dev(s.coeff), dt=s.dt, gravity=s.gravity,
                              bc_layers=s.bc_layers, track_order=False)
    del s
    note(f"affine full size: P={ps.P}")
    for _ in range(2):
        ps.step()
    x, xf = host(ps.x).copy(), host(ps.x_fit).copy()
    c = host(ps.coeff).reshape(3, 27, ps.P).copy()
    ps.sort()
    ps.p2g()
    torch.cuda.synchronize()
    assert ps.status_flags() == 0
    gm = host(ps.grid_mass).astype(np.float64)
    gp = host(ps.grid_mom).astype(np.float64).reshape(3, -1)
    nodes = sample_nodes(gm.reshape(og.nz, og.ny, og.nx), 400, seed=5)
    touch = particles_touching(og, x, nodes)
    M, Q = O.p2g_affine(og, x[:, touch], c[:, :, touch], 27, ps.dt, x_fit=xf[:, touch])
    e_m = rel(gm[nodes], M.ravel()[nodes])
    e_p = rel(gp[:, nodes], Q.reshape(3, -1)[:, nodes])
    note(f"  {nodes.size} nodes, {touch.size} particles: mass {e_m:.2e} momentum {e_p:.2e}")
    assert e_m <= TOL_NORMWISE and e_p <= TOL_NORMWISE
