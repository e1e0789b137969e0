"""Full-size parity: the benchmark workloads, in the launch configuration the benchmark times.

Workloads (seeded, synthetic): the dam break with moving state (128^3 cells, 4,194,304
particles), the falling fluid block (256^3 cells, 16,777,216 particles at 16 per cell) and
the fabric sheet (1,000,000 points with per-point mass and F), all at 27 modes.  One step
runs after the library's autotuner has picked the P2G configuration, as in the benchmark.

The oracle cannot run the whole of these in seconds, so it is run on samples:
* sort: the full permutation and keys, bit for bit (numpy stable argsort);
* P2G: grid mass and momentum at sampled nodes (half of them occupied), from the
  oracle run over every particle whose stencil touches them; plus conservation of mass
  and linear momentum over the whole grid;
* grid update: at the sampled nodes, from the device's grid mass and momentum;
* G2P + advection (+ F): at sampled particles, teacher-forced with the device's grid
  velocity.
The bars are the ones of the parity tests (normwise 1e-5; positions within 2 ulp).
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import polypic_oracle as O
from tests.gpu_util import (TOL_NORMWISE, dev, host, note, oracle_grid, particles_touching, rel,
                            require_gpu, sample_nodes, ulp_ok)

pytestmark = pytest.mark.gpu

CASES = {
    "dambreak_moving_128cube_4194304": (lambda: W.config1_moving(0), 600),
    "fluid_256cube_16777216": (lambda: W.config2_fluid(0), 300),
    "fabric_256cube_1000000": (lambda: W.config2_fabric(0), 600),
}


@pytest.mark.parametrize("case", list(CASES))
def test_full_size_step_sampled(case):
    pp = require_gpu()
    make, n_nodes_sample = CASES[case]
    note(f"full-size step: {case}: generating inputs")
    s = make()
    nm = 27
    note(f"  P={s.P}, running the step")
    g = pp.grid_from_spec(s.grid)
    og = oracle_grid(g)
    ps = pp.ParticleSet(g, nm, dev(s.x), dev(s.coeff[:, :nm]),
                        mass=None if s.mass is None else dev(s.mass),
                        uniform_mass=s.uniform_mass, F=None if s.F is None else dev(s.F),
                        dt=s.dt, gravity=s.gravity, bc_layers=s.bc_layers)
    choice = ps.autotune()          # the benchmark's launch configuration
    note(f"  p2g configuration {tuple(choice)}")
    ps.sort()
    ps.p2g()
    ps.grid_update()
    ps.g2p()
    torch.cuda.synchronize()
    assert ps.status_flags() == 0

    # sort, bit for bit
    note("  oracle sort")
    keys_ref, perm_ref = O.sort_keys(og, s.x)
    perm = host(ps.perm)
    assert np.array_equal(host(ps.keys).view(np.uint32), keys_ref)
    assert np.array_equal(perm, perm_ref)

    gm = host(ps.grid_mass).astype(np.float64)
    gp = host(ps.grid_mom).astype(np.float64).reshape(3, -1)
    gv = host(ps.grid_vel).astype(np.float64).reshape(3, -1)
    m = np.full(s.P, s.uniform_mass) if s.mass is None else s.mass.astype(np.float64)

    # conservation over the whole grid (Eq. 1 and 4 sum to the particle totals)
    assert abs(gm.sum() - m.sum()) <= 1e-5 * m.sum()
    mom = (s.coeff[:, 0, :].astype(np.float64) * m).sum(axis=1)
    scale = (np.abs(s.coeff[:, 0, :].astype(np.float64)) * m).sum(axis=1)
    assert np.all(np.abs(gp.sum(axis=1) - mom) <= 1e-5 * scale), (gp.sum(axis=1), mom)

    # P2G and grid update at sampled nodes
    nodes = sample_nodes(gm.reshape(og.nz, og.ny, og.nx), n_nodes_sample, seed=1)
    touch = particles_touching(og, s.x, nodes)
    note(f"  {nodes.size} sampled nodes, {touch.size} particles touching them")
    M_ref, Q_ref = O.p2g(og, s.x[:, touch], s.coeff[:, :, touch], nm,
                         None if s.mass is None else s.mass[touch], s.uniform_mass)
    assert rel(gm[nodes], M_ref.ravel()[nodes]) <= TOL_NORMWISE
    assert rel(gp[:, nodes], Q_ref.reshape(3, -1)[:, nodes]) <= TOL_NORMWISE
    note("  oracle grid update")
    v_ref = O.grid_update(og, gm.reshape(og.nz, og.ny, og.nx), gp.reshape((3, og.nz, og.ny, og.nx)),
                          s.dt, s.gravity, s.bc_layers).reshape(3, -1)
    assert rel(gv[:, nodes], v_ref[:, nodes]) <= TOL_NORMWISE

    # G2P + advection (+ F) at sampled output slots, teacher-forced with the device grid
    rng = np.random.default_rng(2)
    slots = np.sort(rng.choice(s.P, size=min(8192, s.P), replace=False))
    src = perm[slots]
    F_in = None if s.F is None else s.F[:, src]
    c_ref, x_ref, F_ref = O.g2p(og, gv.reshape((3, og.nz, og.ny, og.nx)), s.x[:, src], nm, s.dt,
                                F_in)
    c_out = host(ps.coeff_next).reshape(3, nm, s.P)[:, :, slots]
    assert rel(c_out, c_ref) <= TOL_NORMWISE
    extent = 1.0 + 4.0 / s.grid.cells[0]
    assert ulp_ok(host(ps.x_next)[:, slots], x_ref, 2, extent)
    if s.F is not None:
        assert rel(host(ps.F_next)[:, slots], F_ref) <= 1e-6
        assert np.array_equal(host(ps.mass_next)[slots], s.mass[src])


def test_full_size_falling_block_impulse():
    """Ten free steps of the 16,777,216-particle falling block (away from every wall).

    P2G conserves linear momentum, the grid update adds dt g to the velocity of every
    occupied node, and the mode-0 G2P coefficient is the W-weighted mean of the node
    velocities, so the particles' total momentum sum_p m_p c_p0 changes by exactly
    M g dt per step (M the total mass); the test allows float32 summation error.
    """
    pp = require_gpu()
    note("full-size impulse: fluid_256cube_16777216: generating inputs")
    s = W.config2_fluid(0)
    g = pp.grid_from_spec(s.grid)
    ps = pp.ParticleSet(g, 27, dev(s.x), dev(s.coeff[:, :27]), dt=s.dt, gravity=s.gravity,
                        bc_layers=s.bc_layers, track_order=False)
    c0 = s.coeff[:, 0, :].astype(np.float64)
    mom0 = c0.sum(axis=1)                 # unit masses
    scale = np.abs(c0).sum(axis=1)
    n_steps = 10
    for k in range(n_steps):
        ps.step()
    torch.cuda.synchronize()
    assert ps.status_flags() == 0
    c = host(ps.coeff[:, 0, :]).astype(np.float64)
    assert np.all(np.isfinite(c))
    expect = mom0 + s.P * np.asarray(s.gravity) * s.dt * n_steps
    note(f"  momentum {c.sum(axis=1)} expected {expect}")
    assert np.all(np.abs(c.sum(axis=1) - expect) <= 1e-5 * scale)
    x = host(ps.x)
    lo = s.grid.origin[1] + 2 * s.grid.dx
    assert x[1].min() > lo + 60 * s.grid.dx   # still far from the floor: no wall acted
