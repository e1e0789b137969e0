"""Active regions on the GPU: the fused scatter flags the 16 x 4 x 4-node regions it lands
in, and the active grid update visits the flagged regions only.

Checked: every node the scatter gave mass or momentum lies in a flagged region, whichever
path the scatter took (LDS bricks for sorted chunks; HBM atomics for chunks of many tiles,
as in input order); the active update equals the dense clearing update on every flagged
region bit for bit (same arithmetic per node), leaves the mass and momentum zero and the
flags reset; and steps whose grid updates are active follow steps with dense updates, for
one scene and for a batch.
"""
import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_util import dev, host, note, rel, require_gpu

pytestmark = pytest.mark.gpu


def region_ids(nx, ny, nz, flat_nodes):
    """Region (16 x 4 x 4 nodes, x fastest, numbered x fastest) of each flat node index."""
    ix = flat_nodes % nx
    iy = (flat_nodes // nx) % ny
    iz = flat_nodes // (nx * ny)
    rx, ry = -(-nx // 16), -(-ny // 4)
    return ((iz // 4) * ry + iy // 4) * rx + ix // 16


def unpack(state, R):
    """Flags of a region state (one uint32 per region)."""
    st = host(state).astype(np.int64)
    assert st.size == R
    return st


def filled_nodes(gm, gp, N):
    m = host(gm).reshape(N)
    q = host(gp).reshape(3, N)
    return np.flatnonzero((m != 0) | (q != 0).any(axis=0))


def make_set(pp, s, n_modes=27, **kw):
    g = pp.grid_from_spec(s.grid)
    args = dict(dt=s.dt, gravity=s.gravity, bc_layers=s.bc_layers)
    args.update(kw)
    ps = pp.ParticleSet(g, n_modes, dev(s.x), dev(s.coeff[:, :n_modes]),
                        mass=None if s.mass is None else dev(s.mass),
                        uniform_mass=s.uniform_mass,
                        F=None if s.F is None else dev(s.F), **args)
    return g, ps


CASES = {
    "config0_sorted": (lambda: W.config0(1), True),
    "config0_input_order": (lambda: W.config0(1), False),    # chunks of many tiles: HBM path
    "fabric_ragged_sorted": (lambda: W.config2_fabric(2, n=64, side=97), True),
    "random_ragged_input_order": (lambda: W.random_scene(5, 40, 20000 + 37), False),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_scatter_flags_cover_every_node_it_fills(case):
    pp = require_gpu()
    make, use_perm = CASES[case]
    s = make()
    g, ps = make_set(pp, s)
    nx, ny, nz = g.nx, g.ny, g.nz
    N = nx * ny * nz
    note(f"active regions, flags cover: {case} P={s.P}")
    ps.sort()
    ps.p2g()
    ps.grid_update()
    ps.region_state.zero_()
    ps.g2p2g(use_perm=use_perm)
    torch.cuda.synchronize()
    assert ps.status_flags() == 0
    R = pp.ops.polypic_region_count(g)
    flags = unpack(ps.region_state, R)
    need = np.unique(region_ids(nx, ny, nz, filled_nodes(ps.grid_mass, ps.grid_mom, N)))
    assert need.size > 0
    unflagged = int((flags[need] == 0).sum())
    assert unflagged == 0, f"{unflagged} regions with mass unflagged"
    note(f"  {need.size} regions filled, {int((flags != 0).sum())} flagged of {flags.size}")
    # flags go where the stencils are: a flagged region is a neighbour of a filled one (a
    # brick or stencil spans at most two regions per axis, one holding a filled node)
    assert (flags != 0).sum() <= 27 * need.size


@pytest.mark.parametrize("case", ["config0_sorted", "random_ragged_input_order"])
def test_active_update_equals_dense_clearing_update(case):
    pp = require_gpu()
    make, use_perm = CASES[case]
    s = make()
    g, ps = make_set(pp, s, dt=1e-3, gravity=(0.0, -9.8, 0.0), bc_layers=1)
    nx, ny, nz = g.nx, g.ny, g.nz
    N = nx * ny * nz
    note(f"active update vs dense: {case}")
    ps.sort()
    ps.p2g()
    ps.grid_update()
    ps.region_state.zero_()
    ps.g2p2g(use_perm=use_perm)
    gm, gp = ps.grid_mass.clone(), ps.grid_mom.clone()
    gv_dense = torch.empty_like(ps.grid_vel)
    pp.ops.polypic_grid_update_clear(g, ps.dt, ps.gravity, ps.bc_layers, gm, gp, gv_dense)
    flags_before = unpack(ps.region_state, pp.ops.polypic_region_count(g))
    ps.grid_vel.fill_(12345.0)
    ps.grid_update_active()
    torch.cuda.synchronize()
    nodes = np.arange(N)
    visited = flags_before[region_ids(nx, ny, nz, nodes)] != 0
    va = host(ps.grid_vel).reshape(3, N)
    vd = host(gv_dense).reshape(3, N)
    assert np.array_equal(va[:, visited], vd[:, visited])
    assert (va[:, ~visited] == 12345.0).all()          # other regions are not touched
    assert float(ps.grid_mass.abs().max()) == 0.0 and float(ps.grid_mom.abs().max()) == 0.0
    assert int(ps.region_state.abs().max()) == 0    # every flag reset


@pytest.mark.parametrize("n_modes", [8, 27])
def test_steps_with_active_updates_follow_dense_steps(n_modes):
    """Six fused steps of a moving scene: ParticleSet.step (the update visits flagged regions
    from the second step on) against the same calls with a dense clearing update."""
    pp = require_gpu()
    s = W.config0(6)
    _, a = make_set(pp, s, n_modes, dt=2e-3)
    _, b = make_set(pp, s, n_modes, dt=2e-3)
    for k in range(6):
        a.step()
        b.sort()
        if k == 0:
            b.p2g()
        b.grid_update(clear=True)
        b.g2p2g(accumulate=True)
        b.swap()
    torch.cuda.synchronize()
    assert a.regions_valid
    assert a.status_flags() == 0 and b.status_flags() == 0
    assert torch.equal(a.order, b.order)
    assert rel(host(a.x), host(b.x)) <= 1e-6
    assert rel(host(a.coeff), host(b.coeff)) <= 1e-5
    assert rel(host(a.grid_mass), host(b.grid_mass)) <= 1e-5


def _batch(pp, seed):
    scenes = W.batched_scenes(seed, n_scenes=5, sizes=(16, 24, 32), p_lo=500, p_hi=2e4)
    grids = [pp.grid_from_spec(sc.grid) for sc in scenes]
    x = np.concatenate([sc.x for sc in scenes], axis=1)
    c = np.concatenate([sc.coeff for sc in scenes], axis=2)
    bs = pp.BatchedParticleSet(grids, [sc.P for sc in scenes], 27, dev(x), dev(c),
                               dt=2e-3, gravity=scenes[0].gravity, bc_layers=1)
    return scenes, grids, bs


def test_batched_flags_cover_every_scene():
    pp = require_gpu()
    scenes, grids, bs = _batch(pp, 3)
    note(f"batched active regions: {[sc.P for sc in scenes]}")
    counts = [pp.ops.polypic_region_count(g) for g in grids]
    assert bs.batch.n_regions == sum(counts)
    bs.step()   # the first step's G2P2G clears densely and flags
    torch.cuda.synchronize()
    assert bs.regions_valid and bs.status_flags() == 0
    flags = unpack(bs.region_state, bs.batch.n_regions)
    begin = np.concatenate([[0], np.cumsum(counts)])
    N = bs.batch.N
    for k, g in enumerate(grids):
        ns = bs.node_slice(k)
        Nk = ns.stop - ns.start
        m = host(bs.grid_mass[ns])
        q = host(bs.grid_mom.reshape(3, N)[:, ns])
        filled = np.flatnonzero((m != 0) | (q != 0).any(axis=0))
        need = np.unique(region_ids(g.nx, g.ny, g.nz, filled)) + begin[k]
        assert need.size > 0 and (flags[need] != 0).all(), k
        assert Nk == g.nx * g.ny * g.nz


def test_batched_steps_with_active_updates_follow_dense_steps():
    """Four batched steps (active updates from the second on) against four steps whose
    updates are dense (the region bookkeeping dropped before each)."""
    pp = require_gpu()
    _, _, a = _batch(pp, 4)
    _, _, b = _batch(pp, 4)
    for _ in range(4):
        a.step()
        b.regions_valid = False
        b.step()
    torch.cuda.synchronize()
    assert a.status_flags() == 0 and b.status_flags() == 0
    assert torch.equal(a.perm, b.perm)
    assert rel(host(a.x), host(b.x)) <= 1e-6
    assert rel(host(a.coeff), host(b.coeff)) <= 1e-5
