"""Full-size parity of the paths the benchmark times, teacher-forced after several steps.

Workloads (seeded, synthetic, 27 modes): the moving dam break (128^3 cells, 4,194,304
particles), the falling fluid block (256^3 cells, 16,777,216 particles) and the fabric
sheet (1,000,000 points with per-point mass and F); the 64-scene batch (25,731,648
particles on 64^3 / 96^3 / 128^3 grids); and one adjoint step of the moving dam break.

The forward sets step as the benchmark does: fused steps (exact re-sort -> grid update ->
G2P + advection fused with the next P2G) after the autotuner has chosen the P2G
configuration; the batch is replayed from its captured graphs.  After k steps the
device state is handed to the oracle (teacher forcing: free-running float32 and float64
trajectories part where a particle crosses a cell switch under different rounding), and
one more step is checked phase by phase:

* the grid the last fused call wrote = the oracle's P2G (Eq. 1, 4, 13) of the state it
  wrote, at sampled nodes, from every particle whose stencil touches them;
* the re-sort = the oracle's stable argsort of the keys, bit for bit (every particle);
* grid update (Eq. 5 + walls) at the sampled nodes, from the device's grid sums;
* G2P + advection (+ F) (Eq. 6-8, section 3.3) at sampled slots, from the device's grid
  velocity;
* the new grid of that fused call = the oracle's P2G of the new state, at sampled nodes.

Bars: normwise 1e-5 on grid sums, velocities and coefficients, 1e-6 on F; positions
within 2 float32 ulp of the domain extent; keys and permutation bit for bit.
The adjoint bar is 1e-4 normwise against the FP64 autograd twin.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import adjoint as A
from oracle import polypic_oracle as O
from tests.gpu_util import (TOL_NORMWISE, dev, host, note, oracle_grid, particles_touching, rel,
                            require_gpu, sample_nodes, ulp_ok)

pytestmark = pytest.mark.gpu

NM = 27
TOL_GRAD = 1e-4


def check_p2g_sampled(og, gm, gp, x, c, mass, uniform_mass, n_nodes, seed, what):
    """Device grid sums (gm (N,), gp (3, N)) against the oracle P2G of (x, c, mass) at
    n_nodes sampled nodes, plus whole-grid conservation of mass and momentum."""
    m = np.full(x.shape[1], uniform_mass) if mass is None else mass.astype(np.float64)
    assert abs(gm.sum() - m.sum()) <= 1e-5 * m.sum(), what
    mom = (c[:, 0, :].astype(np.float64) * m).sum(axis=1)
    scale = (np.abs(c[:, 0, :].astype(np.float64)) * m).sum(axis=1)
    assert np.all(np.abs(gp.sum(axis=1) - mom) <= 1e-5 * scale), (what, gp.sum(axis=1), mom)
    nodes = sample_nodes(gm.reshape(og.nz, og.ny, og.nx), n_nodes, seed=seed)
    touch = particles_touching(og, x, nodes)
    M_ref, Q_ref = O.p2g(og, x[:, touch], c[:, :, touch], c.shape[1],
                         None if mass is None else mass[touch], uniform_mass)
    e_m = rel(gm[nodes], M_ref.ravel()[nodes])
    e_p = rel(gp[:, nodes], Q_ref.reshape(3, -1)[:, nodes])
    note(f"  {what}: {nodes.size} nodes, {touch.size} particles: mass {e_m:.2e} mom {e_p:.2e}")
    assert e_m <= TOL_NORMWISE and e_p <= TOL_NORMWISE, what
    return nodes


def check_g2p_sampled(og, gv, x, F, perm, n_slots, seed, dt, c_out, x_out, F_out, m_out,
                      mass, what, nm=NM):
    """G2P + advection (+ F, mass) at sampled output slots, teacher-forced with the
    device grid velocity gv (3, N); slot i holds particle perm[i] of (x, F, mass)."""
    P = x.shape[1]
    rng = np.random.default_rng(seed)
    slots = np.sort(rng.choice(P, size=min(n_slots, P), replace=False))
    src = perm[slots]
    F_in = None if F is None else F[:, src]
    c_ref, x_ref, F_ref = O.g2p(og, gv.reshape((3, og.nz, og.ny, og.nx)), x[:, src], nm, dt,
                                F_in)
    e_c = rel(c_out[:, :, slots], c_ref)
    note(f"  {what}: {slots.size} slots: coeff {e_c:.2e}")
    assert e_c <= TOL_NORMWISE, what
    extent = (og.nx - 4) * og.dx + 4 * og.dx
    assert ulp_ok(x_out[:, slots], x_ref, 2, extent), what
    if F is not None:
        assert rel(F_out[:, slots], F_ref) <= 1e-6, what
        assert np.array_equal(m_out[slots], mass[src]), what


FORWARD_CASES = {  # (workload, sampled nodes, fused steps before the check, modes)
    "dambreak_moving_128cube_4194304": (lambda: W.config1_moving(0), 400, 5, 27),
    "fluid_256cube_16777216": (lambda: W.config2_fluid(0), 200, 5, 27),
    "fabric_256cube_1000000": (lambda: W.config2_fabric(0), 400, 5, 27),
    # the paper's smallest fluid-only scene size, mode count and time step (section 4,
    # Table 2: about 311 thousand particles, 8 modes, dt = 2e-4)
    "paper_dambreak_moving_64cube_311040_8modes":
        (lambda: W.paper_dambreak_small_moving(0), 400, 10, 8),
}


@pytest.mark.parametrize("case", list(FORWARD_CASES))
def test_fused_steps_teacher_forced(case):
    pp = require_gpu()
    make, n_nodes, k_steps, NM = FORWARD_CASES[case]
    note(f"fused full size: {case}: generating inputs")
    s = make()
    g = pp.grid_from_spec(s.grid)
    og = oracle_grid(g)
    ps = pp.ParticleSet(g, NM, dev(s.x), dev(s.coeff[:, :NM]),
                        mass=None if s.mass is None else dev(s.mass),
                        uniform_mass=s.uniform_mass, F=None if s.F is None else dev(s.F),
                        dt=s.dt, gravity=s.gravity, bc_layers=s.bc_layers, track_order=False)
    choice = ps.autotune()
    note(f"  P={s.P}, p2g configuration {tuple(choice)}; {k_steps} fused steps")
    del s
    for _ in range(k_steps):
        ps.step()
    torch.cuda.synchronize()
    assert ps.status_flags() == 0
    assert ps.grid_current

    # the grid that the last G2P2G wrote: the P2G of the state it wrote
    x = host(ps.x).copy()
    c = host(ps.coeff).reshape(3, NM, ps.P).copy()
    mass = None if ps.mass is None else host(ps.mass).copy()
    F = None if ps.F is None else host(ps.F).copy()
    gm = host(ps.grid_mass).astype(np.float64)
    gp = host(ps.grid_mom).astype(np.float64).reshape(3, -1)
    nodes = check_p2g_sampled(og, gm, gp, x, c, mass, ps.uniform_mass, n_nodes, 1,
                              f"grid after {k_steps} fused steps")

    # one more step, phase by phase: re-sort, grid update, G2P2G
    ps.sort()
    torch.cuda.synchronize()
    keys_ref, perm_ref = O.sort_keys(og, x)
    perm = host(ps.perm)
    assert np.array_equal(host(ps.keys).view(np.uint32), keys_ref)
    assert np.array_equal(perm, perm_ref)
    moved = int(np.count_nonzero(perm != np.arange(ps.P)))
    note(f"  re-sort bit-exact ({moved} slots moved)")
    ps.grid_update()
    torch.cuda.synchronize()
    gv = host(ps.grid_vel).astype(np.float64).reshape(3, -1)
    v_ref = O.grid_update(og, gm.reshape(og.nz, og.ny, og.nx),
                          gp.reshape((3, og.nz, og.ny, og.nx)), ps.dt, ps.gravity,
                          ps.bc_layers).reshape(3, -1)
    assert rel(gv[:, nodes], v_ref[:, nodes]) <= TOL_NORMWISE
    del v_ref
    ps.g2p2g()
    torch.cuda.synchronize()
    assert ps.status_flags() == 0
    c1 = host(ps.coeff_next).reshape(3, NM, ps.P)
    x1 = host(ps.x_next)
    F1 = None if F is None else host(ps.F_next)
    m1 = None if mass is None else host(ps.mass_next)
    check_g2p_sampled(og, gv, x, F, perm, 8192, 2, ps.dt, c1, x1, F1, m1, mass,
                      "G2P half of the next step", nm=NM)
    gm1 = host(ps.grid_mass).astype(np.float64)
    gp1 = host(ps.grid_mom).astype(np.float64).reshape(3, -1)
    check_p2g_sampled(og, gm1, gp1, x1, c1, m1, ps.uniform_mass, n_nodes, 3,
                      "P2G half of the next step")


def test_batched_64_scenes_graph_steps_teacher_forced():
    """The 64-scene batch (25,731,648 particles, 30-bit keys, 4 radix passes, the re-sort's
    separate count scan above 4096 workgroups), stepped as the benchmark steps it: one
    eager step, the autotuner, then replays of the captured graphs.  Then the sort of every
    scene is checked bit for bit, and the grid, update and fused G2P2G on the largest
    scene, the smallest and two more."""
    pp = require_gpu()
    note("batched full size: generating 64 scenes")
    scenes = W.batched_scenes(0)
    grids = [pp.grid_from_spec(s.grid) for s in scenes]
    counts = [s.P for s in scenes]
    P = int(sum(counts))
    s0 = scenes[0]
    x0 = np.concatenate([s.x for s in scenes], axis=1)
    c0 = np.concatenate([s.coeff[:, :NM] for s in scenes], axis=2)
    for s in scenes:
        s.coeff = None
    bs = pp.BatchedParticleSet(grids, counts, NM, dev(x0), dev(c0), dt=s0.dt,
                               gravity=s0.gravity, bc_layers=s0.bc_layers)
    del x0, c0
    note(f"  P={P}: one eager step, autotune, capture, 3 replays")
    bs.step()
    choice = bs.autotune()
    note(f"  batch p2g configuration {tuple(choice)}")
    bs.capture()
    for _ in range(3):
        bs.replay()
    torch.cuda.synchronize()
    assert bs.status_flags() == 0
    assert bs.batch.desc.key_bits > 24     # 4 radix passes, as benchmarked

    order = np.argsort(counts)
    pick = sorted({int(order[-1]), int(order[0]), int(order[len(order) // 2]), 17})
    note(f"  checked scenes {pick}: sizes {[counts[k] for k in pick]}")
    x = host(bs.x).copy()
    c = host(bs.coeff).reshape(3, NM, P)
    gm = host(bs.grid_mass).astype(np.float64)
    gp = host(bs.grid_mom).astype(np.float64).reshape(3, -1)
    N = bs.batch.N
    ogs = [O.grid_from_spec(s.grid) for s in scenes]
    nodes = {}
    for k in pick:
        sl, ns = bs.scene_slice(k), bs.node_slice(k)
        nodes[k] = check_p2g_sampled(ogs[k], gm[ns], gp[:, ns], x[:, sl], c[:, :, sl], None,
                                     1.0, 200, 10 + k, f"scene {k} grid after replays")
    del c

    bs.sort()
    torch.cuda.synchronize()
    perm = host(bs.perm).astype(np.int64)
    keys = host(bs.keys).view(np.uint32)
    mbits = bs.batch.desc.morton_bits
    for k in range(len(scenes)):
        sl = bs.scene_slice(k)
        kref, pref = O.sort_keys(ogs[k], x[:, sl])
        assert np.array_equal(perm[sl] - sl.start, pref.astype(np.int64)), k
        assert np.array_equal(keys[sl], (np.uint32(k) << np.uint32(mbits)) | kref), k
    note("  re-sort of every scene bit-exact")
    bs.grid_update()
    bs.g2p2g()
    torch.cuda.synchronize()
    assert bs.status_flags() == 0
    gv = host(bs.grid_vel).astype(np.float64).reshape(3, -1)
    x1 = host(bs.x_next)
    c1 = host(bs.coeff_next).reshape(3, NM, P)
    gm1 = host(bs.grid_mass).astype(np.float64)
    gp1 = host(bs.grid_mom).astype(np.float64).reshape(3, N)
    for k in pick:
        sl, ns = bs.scene_slice(k), bs.node_slice(k)
        og = ogs[k]
        shp = (og.nz, og.ny, og.nx)
        v_ref = O.grid_update(og, gm[ns].reshape(shp), gp[:, ns].reshape((3,) + shp), bs.dt,
                              bs.gravity, bs.bc_layers).reshape(3, -1)
        assert rel(gv[:, ns][:, nodes[k]], v_ref[:, nodes[k]]) <= TOL_NORMWISE, k
        check_g2p_sampled(og, gv[:, ns], x[:, sl], None, perm[sl] - sl.start, 4096, 20 + k,
                          bs.dt, c1[:, :, sl], x1[:, sl], None, None, None,
                          f"scene {k} G2P half")
        check_p2g_sampled(og, gm1[ns], gp1[:, ns], x1[:, sl], c1[:, :, sl], None, 1.0, 200,
                          30 + k, f"scene {k} P2G half")


def test_adjoint_step_sampled_full_size():
    """One backward step of the moving dam break (4,194,304 particles, 27 modes) after two
    fused steps, with random upstream gradients of the step's outputs.  Teacher-forced
    against the FP64 twin (oracle/adjoint.py):

    * G2P adjoint, dL/dv at sampled nodes: the twin's G2P + advection of every particle
      touching them, differentiated with respect to the (device) grid velocity;
    * grid-update adjoint at sampled nodes, from the device's dL/dv;
    * dL/dx and dL/dc at sampled particles: the twin's G2P of the particle on the device
      grid velocity plus its P2G against the device's dL/dm, dL/dp of the grid.
    """
    pp = require_gpu()
    note("adjoint full size: generating inputs")
    s = W.config1_moving(0)
    g = pp.grid_from_spec(s.grid)
    og = oracle_grid(g)
    ps = pp.ParticleSet(g, NM, dev(s.x), dev(s.coeff[:, :NM]), dt=s.dt, gravity=s.gravity,
                        bc_layers=s.bc_layers, track_order=False)
    P = ps.P
    del s
    for _ in range(2):
        ps.step()
    ps.sort()
    ps.grid_update()
    rng = np.random.default_rng(9)
    gc_up = rng.standard_normal((3, NM, P), dtype=np.float32)   # dL/dc' by output slot
    gx_up = rng.standard_normal((3, P), dtype=np.float32)       # dL/dx' by output slot
    f32 = dict(dtype=torch.float32, device="cuda")
    N = pp.ops.n_nodes(g)
    gvb = torch.empty(3 * N, **f32)
    gmb = torch.empty(N, **f32)
    gpb = torch.empty(3 * N, **f32)
    gx_in = torch.zeros(3, P, **f32)
    gc_in = torch.empty(3, NM, P, **f32)
    st = ps.status
    note(f"  P={P}: adjoint calls")
    pp.ops.polypic_g2p_backward(g, NM, ps.dt, ps.grid_vel, ps.x, dev(gc_up), gvb, gx_in,
                                perm=ps.perm, x_out_grad=dev(gx_up), status_dev=st)
    pp.ops.polypic_grid_update_backward(g, ps.dt, ps.gravity, ps.bc_layers, ps.grid_mass,
                                        ps.grid_mom, gvb, gmb, gpb)
    pp.ops.polypic_p2g_backward(g, NM, ps.x, ps.coeff, gmb, gpb, gc_in, gx_in,
                                uniform_mass=ps.uniform_mass, status_dev=st)
    torch.cuda.synchronize()
    assert ps.status_flags() == 0
    x = host(ps.x).astype(np.float64)
    c = host(ps.coeff).reshape(3, NM, P).astype(np.float64)
    perm = host(ps.perm).astype(np.int64)
    slot_of = np.empty(P, np.int64)
    slot_of[perm] = np.arange(P)
    gm = host(ps.grid_mass).astype(np.float64)
    gp = host(ps.grid_mom).astype(np.float64).reshape(3, -1)
    gv = torch.from_numpy(host(ps.grid_vel).astype(np.float64).reshape(3, -1))
    d_gv = host(gvb).astype(np.float64).reshape(3, -1)
    d_gm = host(gmb).astype(np.float64)
    d_gp = host(gpb).astype(np.float64).reshape(3, -1)
    d_x = host(gx_in).astype(np.float64)
    d_c = host(gc_in).reshape(3, NM, P).astype(np.float64)

    # G2P adjoint at sampled nodes
    nodes = sample_nodes(gm.reshape(og.nz, og.ny, og.nx), 96, seed=4)
    touch = particles_touching(og, x.astype(np.float32), nodes)
    note(f"  dL/dv: {nodes.size} nodes, {touch.size} particles")
    v = gv.clone().requires_grad_(True)
    xo, co = A.g2p(og, v, torch.from_numpy(x[:, touch]), NM, ps.dt)
    sl = slot_of[touch]
    L = ((torch.from_numpy(gc_up[:, :, sl].astype(np.float64)) * co).sum()
         + (torch.from_numpy(gx_up[:, sl].astype(np.float64)) * xo).sum())
    (gv_ref,) = torch.autograd.grad(L, v)
    e_v = rel(d_gv[:, nodes], gv_ref.numpy()[:, nodes])
    note(f"  dL/dv {e_v:.2e}")
    assert e_v <= TOL_GRAD

    # grid-update adjoint at sampled nodes (from the device's dL/dv)
    Mt = torch.from_numpy(gm[nodes]).requires_grad_(True)
    Qt = torch.from_numpy(gp[:, nodes]).requires_grad_(True)
    vt = A.grid_update(og, Mt, Qt, ps.dt, ps.gravity, ps.bc_layers, nodes=torch.from_numpy(nodes))
    gM, gQ = torch.autograd.grad((torch.from_numpy(d_gv[:, nodes]) * vt).sum(), (Mt, Qt))
    e_m, e_q = rel(d_gm[nodes], gM.numpy()), rel(d_gp[:, nodes], gQ.numpy())
    note(f"  grid update adjoint: dL/dm {e_m:.2e} dL/dp {e_q:.2e}")
    assert e_m <= TOL_GRAD and e_q <= TOL_GRAD

    # particle gradients at sampled particles (G2P part + P2G part)
    ps_idx = np.sort(rng.choice(P, size=4096, replace=False))
    xt = torch.from_numpy(x[:, ps_idx]).requires_grad_(True)
    ct = torch.from_numpy(c[:, :, ps_idx]).requires_grad_(True)
    sl = slot_of[ps_idx]
    xo, co = A.g2p(og, gv, xt, NM, ps.dt)
    M, Q = A.p2g(og, xt, ct, NM, None, ps.uniform_mass)
    L = ((torch.from_numpy(gc_up[:, :, sl].astype(np.float64)) * co).sum()
         + (torch.from_numpy(gx_up[:, sl].astype(np.float64)) * xo).sum()
         + (torch.from_numpy(d_gm) * M).sum() + (torch.from_numpy(d_gp) * Q).sum())
    gx_ref, gc_ref = torch.autograd.grad(L, (xt, ct))
    e_x = rel(d_x[:, ps_idx], gx_ref.numpy())
    e_c = rel(d_c[:, :, ps_idx], gc_ref.numpy())
    note(f"  particles: dL/dx {e_x:.2e} dL/dc {e_c:.2e}")
    assert e_x <= TOL_GRAD and e_c <= TOL_GRAD
