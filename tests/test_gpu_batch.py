"""Batched scenes on the GPU: one launch per phase for many independent scenes.

Every scene of a batch is checked against the oracle run on that scene alone
(sort bit-exact; grid and coefficients at the normwise parity bar), and the
batched G2P against the single-scene G2P of the library bit for bit (it is
deterministic).  The graph-captured step is replayed several times with eager
work between the replays, and every replay is checked against an eager step
from the same state.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import polypic_oracle as O
from tests.gpu_util import TOL_NORMWISE, dev, host, note, oracle_grid, rel, require_gpu, ulp_ok

pytestmark = pytest.mark.gpu


def small_batch(seed=0, n=6, empty_at=None):
    scenes = W.batched_scenes(seed, n_scenes=n, sizes=(16, 24, 32), p_lo=500, p_hi=2e4)
    if empty_at is not None:
        s = scenes[empty_at]
        s.x = s.x[:, :0].copy()
        s.coeff = s.coeff[:, :, :0].copy()
    return scenes


def make_set(pp, scenes, n_modes, mass=None, fused=True):
    grids = [pp.grid_from_spec(s.grid) for s in scenes]
    counts = [s.P for s in scenes]
    x = np.concatenate([s.x for s in scenes], axis=1)
    c = np.concatenate([s.coeff[:, :n_modes] for s in scenes], axis=2)
    s0 = scenes[0]
    return pp.BatchedParticleSet(grids, counts, n_modes, dev(x), dev(c),
                                 mass=None if mass is None else dev(mass), dt=s0.dt,
                                 gravity=s0.gravity, bc_layers=s0.bc_layers, fused=fused)


def scene_grid_arrays(bs, k, gm, gp, shape):
    ns = bs.node_slice(k)
    N = bs.batch.N
    return gm[ns].reshape(shape), gp.reshape(3, N)[:, ns].reshape((3,) + tuple(shape))


def test_batched_sort_is_the_per_scene_stable_sort():
    pp = require_gpu()
    scenes = small_batch(0, n=7, empty_at=3)
    note(f"batch sort: {[s.P for s in scenes]}")
    bs = make_set(pp, scenes, 4)
    bs.sort()
    torch.cuda.synchronize()
    assert bs.status_flags() == 0
    perm = host(bs.perm).astype(np.int64)
    keys = host(bs.keys).view(np.uint32)
    mbits = bs.batch.desc.morton_bits
    for k, s in enumerate(scenes):
        sl = bs.scene_slice(k)
        if s.P == 0:
            assert sl.start == sl.stop
            continue
        kref, pref = O.sort_keys(O.grid_from_spec(s.grid), s.x)
        assert np.array_equal(perm[sl] - sl.start, pref.astype(np.int64)), k
        assert np.array_equal(keys[sl], (np.uint32(k) << np.uint32(mbits)) | kref), k


def test_batched_resort_over_steps_equals_full_sort():
    """Five fused steps with a larger dt (particles change cell): every step's batched
    re-sort gives exactly the full batched sort of the same positions, and each scene's
    part is the oracle's stable argsort of that scene."""
    pp = require_gpu()
    scenes = small_batch(8, n=5, empty_at=2)
    note(f"batch re-sort: {[s.P for s in scenes]}")
    bs = make_set(pp, scenes, 8)
    bs.dt = 2e-3
    P = bs.P
    keys_f = torch.empty(P, dtype=torch.int32, device="cuda")
    perm_f = torch.empty(P, dtype=torch.int32, device="cuda")
    ws = torch.empty(pp.ops.polypic_batch_sort_workspace_bytes(bs.batch), dtype=torch.uint8,
                     device="cuda")
    mbits = bs.batch.desc.morton_bits
    changed = 0
    for k in range(5):
        x_before = host(bs.x).copy()
        bs.sort()
        pp.ops.polypic_batch_sort(bs.batch, bs.x, keys_f, perm_f, ws, bs.status)
        torch.cuda.synchronize()
        assert torch.equal(bs.keys, keys_f), k
        assert torch.equal(bs.perm, perm_f), k
        if k > 0:
            changed += int((bs.slot_keys != keys_f[torch.argsort(perm_f.long())]).sum())
        perm = host(bs.perm).astype(np.int64)
        keys = host(bs.keys).view(np.uint32)
        for j, s in enumerate(scenes):
            sl = bs.scene_slice(j)
            if sl.start == sl.stop:
                continue
            kref, pref = O.sort_keys(O.grid_from_spec(s.grid), x_before[:, sl])
            assert np.array_equal(perm[sl] - sl.start, pref.astype(np.int64)), (k, j)
            assert np.array_equal(keys[sl], (np.uint32(j) << np.uint32(mbits)) | kref), (k, j)
        if k == 0:
            bs.p2g()
        bs.grid_update()
        bs.g2p2g()
        bs.swap()
    assert changed > 0
    assert bs.status_flags() == 0


@pytest.mark.parametrize("n_modes", [4, 27])
def test_batched_p2g_every_configuration(n_modes):
    pp = require_gpu()
    scenes = small_batch(1, n=6)
    rng = np.random.default_rng(5)
    mass = (1.0 + 0.5 * rng.random(sum(s.P for s in scenes))).astype(np.float32)
    note(f"batch p2g: n_modes={n_modes} {[s.P for s in scenes]}")
    bs = make_set(pp, scenes, n_modes, mass=mass)
    refs = []
    off = 0
    for s in scenes:
        refs.append(O.p2g(O.grid_from_spec(s.grid), s.x, s.coeff, n_modes, mass[off:off + s.P]))
        off += s.P
    bs.sort()
    configs = [(b, sc, pc, e) for e in (4, 2, 8) for b in (256, 512)
               for sc, pc in ((0, 0), (1, 0), (2, 1), (2, 4))]
    try:
        for cfg in configs:
            pp.ops.polypic_batch_set_config(n_modes, *cfg)
            for use_perm in (True, False):
                bs.p2g(use_perm=use_perm)
                torch.cuda.synchronize()
                gm, gp = host(bs.grid_mass), host(bs.grid_mom)
                for k, (M, Q) in enumerate(refs):
                    m_k, q_k = scene_grid_arrays(bs, k, gm, gp, M.shape)
                    assert rel(m_k, M) <= TOL_NORMWISE, (cfg, use_perm, k)
                    assert rel(q_k, Q) <= TOL_NORMWISE, (cfg, use_perm, k)
        choice = bs.autotune()
        assert (choice.block, choice.schedule, choice.per_cu) in \
            [(b, sc, pc) for b in (256, 512) for sc, pc in ((0, 0), (1, 0), (2, 2), (2, 4), (2, 8))]
        assert choice.brick in (2, 4, 8) and (choice.schedule != 2 or choice.brick == 4)
        gm, gp = host(bs.grid_mass), host(bs.grid_mom)
        for k, (M, Q) in enumerate(refs):
            assert rel(scene_grid_arrays(bs, k, gm, gp, M.shape)[1], Q) <= TOL_NORMWISE
    finally:
        pp.ops.polypic_batch_set_config(n_modes, 256, pp.POLYPIC_SCHED_XCD, 0, 4)
    assert bs.status_flags() == 0


@pytest.mark.parametrize("n_modes", [1, 8, 27])
@pytest.mark.parametrize("fused", [False, True])
def test_batched_step_matches_the_oracle_per_scene(n_modes, fused):
    """One step of every scene against the oracle's step of that scene alone.  Fused
    (polypic_batch_g2p2g), the grid then holds the P2G of the new state: it is compared with
    the oracle's P2G of the state the device wrote, scene by scene."""
    pp = require_gpu()
    scenes = small_batch(2, n=6, empty_at=0)
    note(f"batch step: n_modes={n_modes} fused={fused} {[s.P for s in scenes]}")
    bs = make_set(pp, scenes, n_modes, fused=fused)
    bs.step()
    torch.cuda.synchronize()
    assert bs.status_flags() == 0
    gm, gp = host(bs.grid_mass), host(bs.grid_mom)
    xs, cs = host(bs.x), host(bs.coeff)
    for k, s in enumerate(scenes):
        sl = bs.scene_slice(k)
        og = O.grid_from_spec(s.grid)
        if fused:
            M, Q = O.p2g(og, xs[:, sl], cs[:, :, sl], n_modes)
            m_k, q_k = scene_grid_arrays(bs, k, gm, gp, M.shape)
            assert rel(m_k, M) <= TOL_NORMWISE and rel(q_k, Q) <= TOL_NORMWISE, k
        if s.P == 0:
            continue
        ref = O.step(og, s.x, s.coeff, n_modes, s.dt, s.gravity, s.bc_layers, sort=True)
        if not fused:
            m_k, q_k = scene_grid_arrays(bs, k, gm, gp, ref["grid_mass"].shape)
            assert rel(m_k, ref["grid_mass"]) <= TOL_NORMWISE, k
            assert rel(q_k, ref["grid_mom"]) <= TOL_NORMWISE, k
        assert rel(cs[:, :, sl], ref["coeff"]) <= TOL_NORMWISE, k
        assert ulp_ok(xs[:, sl], ref["x"], 2, 1.0 + 4.0 / s.grid.cells[0]), k


def test_batched_g2p_equals_single_scene_g2p_bitwise():
    """Same grid velocities, same particles: the batched G2P (with F and mass) writes
    exactly what the single-scene G2P writes, scene by scene."""
    pp = require_gpu()
    scenes = small_batch(3, n=5)
    note(f"batch g2p vs single: {[s.P for s in scenes]}")
    bs = make_set(pp, scenes, 27)
    P, N = bs.P, bs.batch.N
    rng = np.random.default_rng(9)
    F = dev((np.eye(3).reshape(9, 1) + 0.01 * rng.standard_normal((9, P))).astype(np.float32))
    m = dev((1.0 + rng.random(P)).astype(np.float32))
    bs.sort()
    bs.p2g()
    bs.grid_update()
    c_b = torch.empty(3, 27, P, device="cuda")
    x_b = torch.empty(3, P, device="cuda")
    F_b = torch.empty(9, P, device="cuda")
    m_b = torch.empty(P, device="cuda")
    pp.ops.polypic_batch_g2p(bs.batch, 27, bs.dt, bs.grid_vel, bs.x, c_b, perm=bs.perm, x_out=x_b,
                             F_in=F, F_out=F_b, mass_in=m, mass_out=m_b, status_dev=bs.status)
    gv = bs.grid_vel.reshape(3, N)
    for k, s in enumerate(scenes):
        sl, ns = bs.scene_slice(k), bs.node_slice(k)
        Pk = sl.stop - sl.start
        g = pp.grid_from_spec(s.grid)
        perm_k = (bs.perm[sl] - sl.start).contiguous()
        c_s = torch.empty(3, 27, Pk, device="cuda")
        x_s = torch.empty(3, Pk, device="cuda")
        F_s = torch.empty(9, Pk, device="cuda")
        m_s = torch.empty(Pk, device="cuda")
        pp.ops.polypic_g2p(g, 27, bs.dt, gv[:, ns].contiguous(), bs.x[:, sl].contiguous(), c_s,
                           perm=perm_k, x_out=x_s, F_in=F[:, sl].contiguous(), F_out=F_s,
                           mass_in=m[sl].contiguous(), mass_out=m_s, status_dev=bs.status)
        torch.cuda.synchronize()
        assert torch.equal(c_b[:, :, sl], c_s), k
        assert torch.equal(x_b[:, sl], x_s), k
        assert torch.equal(F_b[:, sl], F_s), k
        assert torch.equal(m_b[sl], m_s), k
    assert bs.status_flags() == 0


def test_batched_g2p2g_with_mass_matches_single_scene_calls():
    """Same grid velocities, same particles, per-particle masses: the batched fused call writes
    what the single-scene fused call writes, scene by scene (outputs bit for bit; grids at
    the parity bar, the atomic sums being unordered)."""
    pp = require_gpu()
    _check_batched_g2p2g_against_single_calls(pp, small_batch(6, n=5))


def test_batched_g2p2g_scene_chunks_with_ragged_counts():
    """The batched fused kernel gives every workgroup a chunk of 256 slots inside one scene
    (the last chunk of a scene partial): scenes of 0, 1, 255, 256, 257, 513 and 700
    particles, two of them empty, against the single-scene calls."""
    pp = require_gpu()
    scenes = small_batch(12, n=9)
    counts = [700, 0, 1, 255, 256, 257, 0, 513, scenes[8].P]
    for s, k in zip(scenes, counts):
        assert s.P >= k
        s.x = s.x[:, :k].copy()
        s.coeff = s.coeff[:, :, :k].copy()
    _check_batched_g2p2g_against_single_calls(pp, scenes)


def _check_batched_g2p2g_against_single_calls(pp, scenes):
    rng = np.random.default_rng(11)
    P_all = sum(s.P for s in scenes)
    mass = (1.0 + rng.random(P_all)).astype(np.float32)
    note(f"batch g2p2g vs single: {[s.P for s in scenes]}")
    bs = make_set(pp, scenes, 27, mass=mass)
    P, N = bs.P, bs.batch.N
    bs.sort()
    bs.p2g()
    bs.grid_update()
    c_b = torch.empty(3, 27, P, device="cuda")
    x_b = torch.empty(3, P, device="cuda")
    m_b = torch.empty(P, device="cuda")
    gm_b = torch.empty(N, device="cuda")
    gp_b = torch.empty(3 * N, device="cuda")
    pp.ops.polypic_batch_g2p2g(bs.batch, 27, bs.dt, bs.grid_vel, bs.x, x_b, c_b, gm_b, gp_b,
                               perm=bs.perm, mass_in=bs.mass, mass_out=m_b,
                               status_dev=bs.status)
    gv = bs.grid_vel.reshape(3, N)
    for k, s in enumerate(scenes):
        sl, ns = bs.scene_slice(k), bs.node_slice(k)
        Pk = sl.stop - sl.start
        g = pp.grid_from_spec(s.grid)
        Nk = ns.stop - ns.start
        if Pk == 0:  # an empty scene: its grid is cleared and nothing is scattered
            torch.cuda.synchronize()
            assert float(gm_b[ns].abs().max()) == 0.0, k
            continue
        perm_k = (bs.perm[sl] - sl.start).contiguous()
        c_s = torch.empty(3, 27, Pk, device="cuda")
        x_s = torch.empty(3, Pk, device="cuda")
        m_s = torch.empty(Pk, device="cuda")
        gm_s = torch.empty(Nk, device="cuda")
        gp_s = torch.empty(3 * Nk, device="cuda")
        pp.ops.polypic_g2p2g(g, 27, bs.dt, gv[:, ns].contiguous(), bs.x[:, sl].contiguous(),
                             x_s, c_s, gm_s, gp_s, perm=perm_k,
                             mass_in=bs.mass[sl].contiguous(), mass_out=m_s,
                             status_dev=bs.status)
        torch.cuda.synchronize()
        assert torch.equal(c_b[:, :, sl], c_s), k
        assert torch.equal(x_b[:, sl], x_s), k
        assert torch.equal(m_b[sl], m_s), k
        assert rel(host(gm_b[ns]), host(gm_s)) <= TOL_NORMWISE, k
        assert rel(host(gp_b.reshape(3, N)[:, ns]), host(gp_s.reshape(3, Nk))) <= TOL_NORMWISE, k
    assert bs.status_flags() == 0


@pytest.mark.parametrize("fused", [False, True])
def test_graph_replays_match_eager_steps(fused):
    """Capture the two step directions once; replay four steps, each checked against an
    eager step from the same state on a second set, with eager work between replays."""
    pp = require_gpu()
    scenes = small_batch(4, n=6)
    note(f"batch graph replay: fused={fused} {[s.P for s in scenes]}")
    bs = make_set(pp, scenes, 27, fused=fused)
    ref = make_set(pp, scenes, 27, fused=fused)
    bs.step()                     # one eager step first: the capture starts mid-run
    torch.cuda.synchronize()
    bs.capture()
    for it in range(4):
        x0, c0 = bs.x.clone(), bs.coeff.clone()
        ref.x.copy_(x0)
        ref.coeff.copy_(c0)
        ref.invalidate_grid()     # its grid is not of this state: the eager step redoes P2G
        torch.cuda.synchronize()
        bs.replay()
        torch.cuda.synchronize()
        ref.step()
        torch.cuda.synchronize()
        assert rel(host(bs.coeff), host(ref.coeff)) <= TOL_NORMWISE, it
        assert rel(host(bs.x), host(ref.x)) <= 1e-6, it
        assert torch.equal(bs.perm, ref.perm), it
        _ = (bs.x.sum() + bs.coeff.sum()).item()  # eager work between replays
    assert bs.status_flags() == 0 and ref.status_flags() == 0


def test_out_of_range_particle_flags_and_stays_in_its_scene():
    pp = require_gpu()
    scenes = small_batch(5, n=4)
    s = scenes[1]
    s.x = s.x.copy()
    s.x[0, 0] = -5.0                              # far outside its grid
    note("batch out-of-range particle")
    bs = make_set(pp, scenes, 4)
    bs.sort()
    torch.cuda.synchronize()
    assert bs.status_flags() & 1
    perm = host(bs.perm)
    for k in range(len(scenes)):
        sl = bs.scene_slice(k)
        assert np.array_equal(np.sort(perm[sl]), np.arange(sl.start, sl.stop)), k
    # P2G of the other scenes is unaffected
    bs.p2g()
    torch.cuda.synchronize()
    gm, gp = host(bs.grid_mass), host(bs.grid_mom)
    for k in (0, 2, 3):
        sc = scenes[k]
        M, Q = O.p2g(O.grid_from_spec(sc.grid), sc.x, sc.coeff, 4)
        m_k, q_k = scene_grid_arrays(bs, k, gm, gp, M.shape)
        assert rel(m_k, M) <= TOL_NORMWISE and rel(q_k, Q) <= TOL_NORMWISE, k


@pytest.mark.parametrize("n_modes", [4, 27])
def test_fused_p2g_does_not_fold_across_a_scene_boundary(n_modes):
    """Two scenes of 129 particles, each particle in its own 4^3-node tile, so that the
    first workgroup's chunk holds more than 64 runs before the scene boundary.  Scene 0's
    last particle (slot 128) and scene 1's first (slot 129) share their local base node
    and form one lane pair of the fused kernel's P2G half.  They belong to different
    grids, so their node values must not be folded together: every scene's grid equals
    the oracle's P2G (Eq. 1, 4, 13) of that scene's new state, and its mass sums to the
    scene's particle count."""
    pp = require_gpu()
    n = 32
    gs = W.cubic_grid(n)
    og = O.grid_from_spec(gs)
    tiles = np.array([(tx, ty, tz) for tz in range(8) for ty in range(8) for tx in range(8)]).T
    bases = 4 * tiles + 1
    order = np.argsort(O.morton_key(bases), kind="stable")
    q = order[300]
    pick = [np.concatenate([order[:128], [q]]), np.concatenate([[q], order[301:429]])]
    rng = np.random.default_rng(11)
    scenes = []
    for k, sel in enumerate(pick):
        x = ((bases[:, sel] + 1.25) * gs.dx).astype(np.float32)   # t = 1/4 on every axis
        c = np.zeros((3, 27, x.shape[1]), np.float32)
        c[:, 0] = rng.standard_normal((3, x.shape[1]))
        c[:, 1:] = 0.1 * rng.standard_normal((3, 26, x.shape[1]))
        scenes.append(W.Scene(f"boundary{k}", gs, x, c, None, 1.0, dt=0.0,
                              gravity=(0.0, 0.0, 0.0), bc_layers=0))
    note(f"batch fused scene boundary: n_modes={n_modes}")
    bs = make_set(pp, scenes, n_modes)
    bs.sort()
    perm = host(bs.perm)
    assert perm[128] == 128 and perm[129] == 129      # the boundary pair, as constructed
    bs.p2g()
    bs.grid_update()
    bs.g2p2g()
    torch.cuda.synchronize()
    assert bs.status_flags() == 0
    x1 = host(bs.x_next)
    c1 = host(bs.coeff_next).reshape(3, n_modes, bs.P)
    gm, gp = host(bs.grid_mass), host(bs.grid_mom)
    for k in range(2):
        sl = bs.scene_slice(k)
        M_ref, Q_ref = O.p2g(og, x1[:, sl], c1[:, :, sl], n_modes)
        M, Q = scene_grid_arrays(bs, k, gm, gp, M_ref.shape)
        assert abs(float(M.sum()) - 129.0) <= 1e-4, (k, float(M.sum()))
        assert rel(M, M_ref) <= TOL_NORMWISE, k
        assert rel(Q, Q_ref) <= TOL_NORMWISE, k
