"""C-ABI contract checks that need no GPU: the library loads, exports every entry
point that include/polypic.h declares, and rejects bad arguments on the host
with the documented status codes before touching the device."""
import ctypes
import os
import re

import pytest

from paper_2308_01060_amd import _lib

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "polypic.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(polypic_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = _lib.load()
    names = declared_functions()
    assert len(names) >= 7
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.EXPORTED)


def test_status_strings_and_version():
    lib = _lib.load()
    assert lib.polypic_version() >= 100
    assert _lib.strerror(0) == "ok"
    assert "workspace" in _lib.strerror(4)
    assert _lib.strerror(99) == "unknown status code"


def grid(nx=36, ny=36, nz=36, dx=1 / 32):
    g = _lib.polypic_grid()
    g.nx, g.ny, g.nz = nx, ny, nz
    g.dx = dx
    g.inv_dx = 1 / dx
    return g


def test_workspace_query():
    lib = _lib.load()
    out = ctypes.c_size_t(0)
    g = grid()
    assert lib.polypic_sort_workspace_bytes(ctypes.byref(g), 32768, ctypes.byref(out)) == 0
    assert out.value >= 2 * 32768 * 4
    assert lib.polypic_sort_workspace_bytes(ctypes.byref(g), -1, ctypes.byref(out)) == 1
    assert lib.polypic_sort_workspace_bytes(None, 10, ctypes.byref(out)) == 1
    big = grid(2000, 36, 36)
    assert lib.polypic_sort_workspace_bytes(ctypes.byref(big), 10, ctypes.byref(out)) == 5


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation


def p2g_call(g, P=10, n_modes=4, x=FAKE, mass=None, umass=1.0, coeff=FAKE, perm=None, keys=None,
             ws=None, ws_bytes=0, gm=FAKE, gp=FAKE, acc=0):
    lib = _lib.load()
    return lib.polypic_p2g(ctypes.byref(g), P, n_modes, x, mass, umass, coeff, perm, keys, ws,
                           ws_bytes, gm, gp, acc, None, None)


@pytest.mark.parametrize("n_modes", [0, 2, 5, 9, 26, 28])
def test_p2g_rejects_bad_mode_count(n_modes):
    assert p2g_call(grid(), n_modes=n_modes) == _lib.POLYPIC_EINVAL


def test_p2g_rejects_null_and_bad_sizes():
    g = grid()
    assert p2g_call(g, x=None) == 1
    assert p2g_call(g, gm=None) == 1
    assert p2g_call(g, P=-5) == 1
    assert p2g_call(g, P=1 << 31) == 1
    assert p2g_call(grid(2, 36, 36)) == 1
    assert p2g_call(grid(dx=-1.0)) == 1
    assert p2g_call(g, umass=float("nan")) == 1
    # sorted path: keys need perm and a workspace of the queried size
    assert p2g_call(g, keys=FAKE, perm=None, ws=FAKE, ws_bytes=1 << 20) == 1
    assert p2g_call(g, keys=FAKE, perm=FAKE, ws=None) == 1
    assert p2g_call(g, keys=FAKE, perm=FAKE, ws=FAKE, ws_bytes=8) == _lib.POLYPIC_ENOSPACE


def test_p2g_workspace_query():
    lib = _lib.load()
    out = ctypes.c_size_t(0)
    g = grid(132, 132, 132, 1 / 128)
    assert lib.polypic_p2g_workspace_bytes(ctypes.byref(g), 4194304, ctypes.byref(out)) == 0
    tiles = (129 // 4 + 1) ** 3
    assert out.value >= 4 + 4 * tiles
    assert lib.polypic_p2g_workspace_bytes(ctypes.byref(g), 10, ctypes.byref(out)) == 0
    assert out.value <= 1024


def test_g2p_rejects_bad_arguments():
    lib = _lib.load()
    g = grid()
    args = lambda **k: dict(dict(P=10, nr=4, dt=1e-4, gv=FAKE, x=FAKE, perm=None, xo=None,  # noqa
                                 co=FAKE, Fi=None, Fo=None, mi=None, mo=None), **k)

    def call(**k):
        a = args(**k)
        return lib.polypic_g2p(ctypes.byref(g), a["P"], a["nr"], a["dt"], a["gv"], a["x"],
                               a["perm"], a["xo"], a["co"], a["Fi"], a["Fo"], a["mi"], a["mo"],
                               None, None)

    assert call(nr=3) == 1
    assert call(gv=None) == 1
    assert call(co=None) == 1
    assert call(Fi=FAKE) == 1       # F_in without F_out
    assert call(mo=FAKE) == 1       # mass_out without mass_in
    assert call(dt=float("inf")) == 1
    assert call(P=0, gv=None, x=None, co=None) == 0  # nothing to do, nothing enqueued


def test_grid_update_and_sort_reject_bad_arguments():
    lib = _lib.load()
    g = grid()
    grav = (ctypes.c_float * 3)(0.0, -9.8, 0.0)
    assert lib.polypic_grid_update(ctypes.byref(g), 1e-4, None, 1, FAKE, FAKE, FAKE, None) == 1
    assert lib.polypic_grid_update(ctypes.byref(g), 1e-4, grav, -1, FAKE, FAKE, FAKE, None) == 1
    assert lib.polypic_grid_update(ctypes.byref(g), 1e-4, grav, 1, None, FAKE, FAKE, None) == 1
    far = lambda k: ctypes.c_void_p(0x10000000 + k * 0x1000000)  # noqa: E731  disjoint, fake
    clear = lib.polypic_grid_update_clear
    assert clear(ctypes.byref(g), 1e-4, None, 1, far(0), far(1), far(2), None) == 1
    assert clear(ctypes.byref(g), 1e-4, grav, -1, far(0), far(1), far(2), None) == 1
    assert clear(ctypes.byref(g), float("nan"), grav, 1, far(0), far(1), far(2), None) == 1
    assert clear(ctypes.byref(g), 1e-4, grav, 1, None, far(1), far(2), None) == 1
    assert clear(ctypes.byref(g), 1e-4, grav, 1, far(0), None, far(2), None) == 1
    assert clear(ctypes.byref(g), 1e-4, grav, 1, far(0), far(1), far(1), None) == 1  # aliasing
    assert clear(None, 1e-4, grav, 1, far(0), far(1), far(2), None) == 1
    assert lib.polypic_sort(ctypes.byref(g), 100, FAKE, FAKE, FAKE, FAKE, 16, None, None) == 4
    assert lib.polypic_sort(ctypes.byref(g), 100, None, FAKE, FAKE, FAKE, 1 << 20, None,
                            None) == 1
    assert lib.polypic_sort(ctypes.byref(g), 0, None, None, None, None, 0, None, None) == 0


def test_p2g_config_table_validation():
    lib = _lib.load()
    path, block, sched, per_cu, brick = (ctypes.c_int32(0) for _ in range(5))
    refs = [ctypes.byref(v) for v in (path, block, sched, per_cu, brick)]
    assert lib.polypic_set_p2g_config(5, 0, 512, 0, 0, 4) == 1         # bad n_modes
    assert lib.polypic_set_p2g_config(27, 7, 512, 0, 0, 4) == 1        # bad path
    assert lib.polypic_set_p2g_config(27, 0, 300, 0, 0, 4) == 1        # bad block
    assert lib.polypic_set_p2g_config(27, 0, 256, 3, 0, 4) == 1        # bad schedule
    assert lib.polypic_set_p2g_config(27, 0, 256, 2, 0, 4) == 1        # persistent needs per_cu
    assert lib.polypic_set_p2g_config(27, 0, 256, 2, 65, 4) == 1
    for bad in (0, 1, 3, 16):                                           # brick edge 2, 4 or 8
        assert lib.polypic_set_p2g_config(27, 0, 256, 0, 0, bad) == 1
    assert lib.polypic_set_p2g_config(8, _lib.POLYPIC_P2G_BRICKS, 256, _lib.POLYPIC_SCHED_XCD,
                                      0, 8) == 0
    assert lib.polypic_get_p2g_config(8, *refs) == 0
    assert (path.value, block.value, sched.value, per_cu.value, brick.value) == (
        _lib.POLYPIC_P2G_BRICKS, 256, _lib.POLYPIC_SCHED_XCD, 0, 8)
    assert lib.polypic_set_p2g_config(8, 0, 512, _lib.POLYPIC_SCHED_PERSISTENT, 4, 2) == 0
    assert lib.polypic_get_p2g_config(8, *refs) == 0
    assert (sched.value, per_cu.value, brick.value) == (_lib.POLYPIC_SCHED_PERSISTENT, 4, 2)
    assert lib.polypic_set_p2g_config(8, _lib.POLYPIC_P2G_DEFAULT, 512, 0, 0, 4) == 0
    assert lib.polypic_get_p2g_config(8, *refs) == 0
    assert path.value == _lib.POLYPIC_P2G_DEFAULT and brick.value == 4
    # fused G2P2G: lane group and chunk order
    lg = ctypes.c_int32(0)
    assert lib.polypic_set_g2p2g_config(5, 2, 0) == 1                   # bad n_modes
    assert lib.polypic_set_g2p2g_config(27, 3, 0) == 1                  # bad lane group
    assert lib.polypic_set_g2p2g_config(27, 2, _lib.POLYPIC_SCHED_PERSISTENT) == 1
    assert lib.polypic_set_g2p2g_config(27, 4, _lib.POLYPIC_SCHED_XCD) == 0
    assert lib.polypic_get_g2p2g_config(27, ctypes.byref(lg), ctypes.byref(sched)) == 0
    assert (lg.value, sched.value) == (4, _lib.POLYPIC_SCHED_XCD)
    assert lib.polypic_set_g2p2g_config(27, -1, -1) == 0
    assert lib.polypic_get_g2p2g_config(27, ctypes.byref(lg), ctypes.byref(sched)) == 0
    assert (lg.value, sched.value) == (2, _lib.POLYPIC_SCHED_LINEAR)
    assert lib.polypic_get_g2p2g_config(27, ctypes.byref(lg), None) == 1
    # G2P schedule
    assert lib.polypic_set_g2p_schedule(2) == 1
    assert lib.polypic_set_g2p_schedule(_lib.POLYPIC_SCHED_XCD) == 0
    assert lib.polypic_get_g2p_schedule(ctypes.byref(sched)) == 0 and sched.value == 1
    assert lib.polypic_set_g2p_schedule(_lib.POLYPIC_SCHED_LINEAR) == 0
    # batched P2G configuration
    assert lib.polypic_batch_set_config(27, 384, 0, 0, 4) == 1
    assert lib.polypic_batch_set_config(27, 256, 2, 0, 4) == 1
    assert lib.polypic_batch_set_config(27, 256, 0, 0, 6) == 1
    assert lib.polypic_batch_get_config(27, *refs[1:]) == 0
    assert (block.value, sched.value, brick.value) == (256, _lib.POLYPIC_SCHED_XCD, 4)  # default
    assert lib.polypic_batch_set_config(4, 512, _lib.POLYPIC_SCHED_PERSISTENT, 8, 2) == 0
    assert lib.polypic_batch_get_config(4, *refs[1:]) == 0
    assert (block.value, sched.value, per_cu.value, brick.value) == (512, 2, 8, 2)
    assert lib.polypic_batch_set_config(4, 256, _lib.POLYPIC_SCHED_XCD, 0, 4) == 0


def scene(g, p_off, n, node_off):
    s = _lib.polypic_scene()
    s.grid = g
    s.p_offset, s.n_particles, s.node_offset = p_off, n, node_off
    return s


def test_region_count_and_active_update_arguments():
    """Active regions: 16 x 4 x 4-node boxes, partial at the upper ends; the active update
    checks its arguments as the clearing update does, and needs the flags."""
    lib = _lib.load()
    out = ctypes.c_int64(0)
    for dims in ((36, 36, 36), (3, 3, 3), (16, 4, 4), (17, 5, 9), (132, 132, 132),
                 (260, 260, 260), (1026, 3, 1026)):
        assert lib.polypic_region_count(ctypes.byref(grid(*dims)), ctypes.byref(out)) == 0
        nx, ny, nz = dims
        assert out.value == -(-nx // 16) * -(-ny // 4) * -(-nz // 4), dims
    assert lib.polypic_region_count(ctypes.byref(grid(2, 36, 36)), ctypes.byref(out)) == 1
    assert lib.polypic_region_count(ctypes.byref(grid()), None) == 1
    g = grid()
    grav = (ctypes.c_float * 3)(0.0, -9.8, 0.0)
    far = lambda k: ctypes.c_void_p(0x10000000 + k * 0x1000000)  # noqa: E731  disjoint, fake
    act = lib.polypic_grid_update_active
    assert act(ctypes.byref(g), 1e-4, grav, 1, far(0), far(1), far(2), None, None) == 1
    assert act(ctypes.byref(g), 1e-4, None, 1, far(0), far(1), far(2), far(3), None) == 1
    assert act(ctypes.byref(g), 1e-4, grav, -1, far(0), far(1), far(2), far(3), None) == 1
    assert act(ctypes.byref(g), float("inf"), grav, 1, far(0), far(1), far(2), far(3), None) == 1
    assert act(ctypes.byref(g), 1e-4, grav, 1, None, far(1), far(2), far(3), None) == 1
    assert act(ctypes.byref(g), 1e-4, grav, 1, far(0), far(1), far(0), far(3), None) == 1
    assert act(None, 1e-4, grav, 1, far(0), far(1), far(2), far(3), None) == 1


def test_batch_plan_validation():
    """Every check that polypic_batch_plan makes before touching the device."""
    lib = _lib.load()
    g = grid(36, 36, 36)
    nn = 36 ** 3
    out = ctypes.c_size_t(0)
    assert lib.polypic_batch_table_bytes(0, ctypes.byref(out)) == 1
    assert lib.polypic_batch_table_bytes(65537, ctypes.byref(out)) == 1
    assert lib.polypic_batch_table_bytes(3, ctypes.byref(out)) == 0 and out.value >= 3 * 64
    table_bytes = out.value
    b = _lib.polypic_batch()

    def plan(scenes, n_total=3 * nn, tb=table_bytes, table=FAKE):
        arr = (_lib.polypic_scene * len(scenes))(*scenes)
        return lib.polypic_batch_plan(arr, len(scenes), n_total, table, tb, ctypes.byref(b), None)

    ok = [scene(g, 0, 10, 0), scene(g, 10, 0, nn), scene(g, 10, 5, 2 * nn)]
    assert plan(ok, table=None) == 1
    assert plan(ok, tb=8) == _lib.POLYPIC_ENOSPACE
    assert plan([scene(g, 0, 10, 0), scene(g, 11, 5, nn)]) == 1        # gap in particle ranges
    assert plan([scene(g, 1, 10, 0)]) == 1                             # does not start at 0
    assert plan([scene(g, 0, -1, 0)]) == 1                             # negative count
    assert plan([scene(g, 0, 10, 0), scene(g, 10, 5, nn - 1)]) == 1    # overlapping nodes
    assert plan([scene(g, 0, 10, 0), scene(g, 10, 5, 2 * nn + 1)]) == 1  # beyond n_nodes_total
    assert plan([scene(grid(2, 36, 36), 0, 10, 0)]) == 1               # bad grid
    # scene index bits + Morton bits above 32: 1026-node grids need 30 Morton bits
    big = grid(1026, 1026, 1026)
    nb = 1026 ** 3
    many = [scene(big, 0, 0, k * nb) for k in range(8)]      # 3 scene bits + 30 Morton bits
    assert plan(many, n_total=8 * nb, tb=1 << 20) == _lib.POLYPIC_ENOTSUP


def test_batch_calls_reject_unplanned_descriptors():
    lib = _lib.load()
    b = _lib.polypic_batch()               # zeroed: no table, wrong seal
    assert lib.polypic_batch_p2g(ctypes.byref(b), 27, FAKE, None, 1.0, FAKE, None, FAKE, FAKE, 0,
                                 None, None) == 1
    b.n_scenes, b.table, b.P, b.N = 1, 0x1000, 10, 100   # filled by hand: the seal does not match
    assert lib.polypic_batch_p2g(ctypes.byref(b), 27, FAKE, None, 1.0, FAKE, None, FAKE, FAKE, 0,
                                 None, None) == 1
    grav = (ctypes.c_float * 3)(0.0, -9.8, 0.0)
    assert lib.polypic_batch_grid_update(ctypes.byref(b), 1e-4, grav, 1, FAKE, FAKE, FAKE,
                                         None) == 1
    assert lib.polypic_batch_g2p(ctypes.byref(b), 27, 1e-4, FAKE, FAKE, None, None, FAKE, None,
                                 None, None, None, None, None) == 1
    assert lib.polypic_batch_g2p2g(ctypes.byref(b), 27, 1e-4, FAKE, FAKE, None, FAKE, FAKE,
                                   None, None, None, None, 1.0, FAKE, FAKE, 0, None, None,
                                   None) == 1
    assert lib.polypic_batch_grid_update_active(ctypes.byref(b), 1e-4, grav, 1, FAKE, FAKE, FAKE,
                                                FAKE, None) == 1
    out = ctypes.c_size_t(0)
    assert lib.polypic_batch_sort_workspace_bytes(ctypes.byref(b), ctypes.byref(out)) == 1
    assert lib.polypic_batch_sort(None, FAKE, FAKE, FAKE, FAKE, 1 << 20, None, None) == 1
    assert lib.polypic_batch_sort_update(ctypes.byref(b), FAKE, FAKE, ctypes.c_void_p(0x2000),
                                         FAKE, FAKE, 1 << 30, None, None) == 1
    assert lib.polypic_batch_sort_update_workspace_bytes(ctypes.byref(b), ctypes.byref(out)) == 1


def test_backward_entry_points_reject_bad_arguments():
    lib = _lib.load()
    g = grid()
    grav = (ctypes.c_float * 3)(0.0, -9.8, 0.0)

    def g2pb(P=10, nr=4, dt=1e-4, gv=FAKE, x=FAKE, perm=None, gco=FAKE, gxo=None, gvb=FAKE,
             gxi=FAKE):
        return lib.polypic_g2p_backward(ctypes.byref(g), P, nr, dt, gv, x, perm, gco, gxo, gvb, 0,
                                        gxi, None, None)

    assert g2pb(nr=5) == 1
    assert g2pb(gv=None) == 1
    assert g2pb(gco=None) == 1
    assert g2pb(gvb=None) == 1
    assert g2pb(gxi=None) == 1
    assert g2pb(dt=float("nan")) == 1
    assert g2pb(P=-1) == 1

    def gub(gv=FAKE, gm=FAKE, gp=FAKE, gmb=FAKE, gpb=FAKE, bc=1, gr=grav):
        return lib.polypic_grid_update_backward(ctypes.byref(g), 1e-4, gr, bc, gm, gp, gv, gmb,
                                                gpb, None)

    assert gub(gr=None) == 1
    assert gub(bc=-2) == 1
    assert gub(gm=None) == 1
    assert gub(gv=None) == 1
    assert gub(gpb=None) == 1
    assert lib.polypic_grid_update_backward(None, 1e-4, grav, 1, FAKE, FAKE, FAKE, FAKE, FAKE,
                                            None) == 1

    def p2gb(P=10, nr=4, x=FAKE, mass=None, umass=1.0, c=FAKE, gmb=FAKE, gpb=FAKE, cg=FAKE,
             xg=FAKE, mg=None):
        return lib.polypic_p2g_backward(ctypes.byref(g), P, nr, x, mass, umass, c, None, gmb, gpb,
                                        cg, xg, mg, None, None)

    assert p2gb(nr=26) == 1
    assert p2gb(x=None) == 1
    assert p2gb(gmb=None) == 1
    assert p2gb(cg=None) == 1
    assert p2gb(xg=None) == 1
    assert p2gb(umass=float("inf")) == 1
    assert p2gb(P=0, x=None, c=None, cg=None, xg=None) == 0


def test_sort_update_rejects_bad_arguments():
    lib = _lib.load()
    g = grid()
    out = ctypes.c_size_t(0)
    assert lib.polypic_sort_update_workspace_bytes(ctypes.byref(g), 1000, ctypes.byref(out)) == 0
    need = out.value
    assert need >= 24 * 1000
    other = ctypes.c_void_p(0x2000)
    call = lambda x=FAKE, kp=FAKE, ko=other, pm=FAKE, ws=FAKE, wsb=need: lib.polypic_sort_update(  # noqa
        ctypes.byref(g), 1000, x, kp, ko, pm, ws, wsb, None, None)
    assert call(kp=None) == 1
    assert call(x=None) == 1
    assert call(ko=FAKE) == 1                 # keys_prev aliases keys_out
    assert call(wsb=need - 1) == _lib.POLYPIC_ENOSPACE
    assert lib.polypic_sort_update(ctypes.byref(g), 0, None, None, None, None, None, 0, None,
                                   None) == 0


def test_g2p2g_rejects_bad_arguments():
    lib = _lib.load()
    g = grid()
    far = lambda k: ctypes.c_void_p(0x10000000 + k * 0x1000000)  # noqa: E731  disjoint, fake
    gv, x, xo, co, gm, gp = (far(k) for k in range(6))

    def call(n_modes=27, dt=1e-4, gv=gv, x=x, perm=None, xo=xo, co=co, fi=None, fo=None,
             mi=None, mo=None, um=1.0, gm=gm, gp=gp, acc=0):
        return lib.polypic_g2p2g(ctypes.byref(g), 10, n_modes, dt, gv, x, perm, xo, co, fi, fo,
                                 mi, mo, um, gm, gp, acc, None, None, None)
    assert call(n_modes=5) == 1
    assert call(dt=float("nan")) == 1
    assert call(xo=None) == 1                   # the scatter needs the advected positions
    assert call(co=None) == 1
    assert call(gm=None) == 1 and call(gp=None) == 1
    assert call(fi=far(7)) == 1                 # F_in without F_out
    assert call(mo=far(8)) == 1                 # mass_out without mass_in
    assert call(um=float("inf")) == 1
    assert call(xo=x) == 1                      # x_out overlaps x_in
    assert call(gm=gv) == 1                     # the next grid overlaps grid_vel
    assert call(gp=ctypes.c_void_p(0x10000000 + 4 * 0x1000000 + 4)) == 1  # grid_mom over grid_mass
    assert call(fi=far(7), fo=far(7)) == 1      # F_out overlaps F_in
    assert call(acc=1, xo=None) == 1            # accumulating changes none of the checks
    assert call(acc=1, gm=gv) == 1


def test_permutation_calls_reject_bad_arguments():
    lib = _lib.load()
    far = lambda k: ctypes.c_void_p(0x10000000 + k * 0x1000000)  # noqa: E731  disjoint, fake
    src, dst, idx = far(0), far(1), far(2)
    assert lib.polypic_gather_rows(None, dst, idx, 3, 10, None) == 1
    assert lib.polypic_gather_rows(src, None, idx, 3, 10, None) == 1
    assert lib.polypic_gather_rows(src, dst, None, 3, 10, None) == 1
    assert lib.polypic_gather_rows(src, dst, idx, -1, 10, None) == 1
    assert lib.polypic_gather_rows(src, dst, idx, 3, -1, None) == 1
    assert lib.polypic_gather_rows(src, dst, idx, 3, 2**31, None) == 1
    assert lib.polypic_gather_rows(src, ctypes.c_void_p(0x10000000 + 100), idx, 3, 10, None) == 1
    assert lib.polypic_gather_rows(None, None, None, 0, 10, None) == 0   # nothing to move
    assert lib.polypic_gather_rows(None, None, None, 3, 0, None) == 0
    assert lib.polypic_scatter_rows(None, dst, idx, 3, 10, None) == 1
    assert lib.polypic_scatter_rows(src, dst, None, 3, 10, None) == 1
    assert lib.polypic_scatter_rows(src, ctypes.c_void_p(0x10000000 + 100), idx, 3, 10, None) == 1
    assert lib.polypic_scatter_rows(None, None, None, 3, 0, None) == 0
    assert lib.polypic_invert_permutation(None, dst, 10, None) == 1
    assert lib.polypic_invert_permutation(idx, None, 10, None) == 1
    assert lib.polypic_invert_permutation(idx, ctypes.c_void_p(0x10000000 + 2 * 0x1000000 + 8),
                                          10, None) == 1             # inv overlaps perm
    assert lib.polypic_invert_permutation(idx, dst, -5, None) == 1
    assert lib.polypic_invert_permutation(None, None, 0, None) == 0


def test_sort_noalloc_host_checks():
    """The allocation-free sort rejects more than POLYPIC_SORT_NOALLOC_MAX_P particles with
    POLYPIC_ENOSPACE, and null arrays with POLYPIC_EINVAL, before touching the device."""
    lib = _lib.load()
    g = grid()
    cap = _lib.POLYPIC_SORT_NOALLOC_MAX_P
    text = open(HEADER).read()
    assert f"#define POLYPIC_SORT_NOALLOC_MAX_P {cap}" in text
    assert lib.polypic_sort_noalloc(ctypes.byref(g), cap + 1, FAKE, FAKE, FAKE, None,
                                    None) == _lib.POLYPIC_ENOSPACE
    assert lib.polypic_sort_noalloc(ctypes.byref(g), 10, None, FAKE, FAKE, None,
                                    None) == _lib.POLYPIC_EINVAL
    assert lib.polypic_sort_noalloc(ctypes.byref(g), 10, FAKE, FAKE, None, None,
                                    None) == _lib.POLYPIC_EINVAL
    assert lib.polypic_sort_noalloc(ctypes.byref(g), -1, FAKE, FAKE, FAKE, None,
                                    None) == _lib.POLYPIC_EINVAL
    assert lib.polypic_sort_noalloc(None, 10, FAKE, FAKE, FAKE, None, None) == 1
    assert lib.polypic_sort_noalloc(ctypes.byref(g), 0, None, None, None, None, None) == 0
    # the static workspace covers the full sort's workspace at the cap
    out = ctypes.c_size_t(0)
    assert lib.polypic_sort_workspace_bytes(ctypes.byref(g), cap, ctypes.byref(out)) == 0
    assert out.value <= 18 << 20


def test_mac_calls_reject_bad_arguments_on_the_host():
    """The staggered-grid calls validate like their collocated counterparts."""
    lib = _lib.load()
    g = grid()
    g3 = (ctypes.c_float * 3)(0.0, -9.8, 0.0)
    # P2G: bad mode count, null face arrays, null inputs with P > 0, bad P, bad grid
    assert lib.polypic_mac_p2g(ctypes.byref(g), 10, 5, FAKE, None, 1.0, FAKE, None, FAKE, FAKE,
                               0, None, None) == _lib.POLYPIC_EINVAL
    assert lib.polypic_mac_p2g(ctypes.byref(g), 10, 4, FAKE, None, 1.0, FAKE, None, None, FAKE,
                               0, None, None) == _lib.POLYPIC_EINVAL
    assert lib.polypic_mac_p2g(ctypes.byref(g), 10, 4, None, None, 1.0, FAKE, None, FAKE, FAKE,
                               0, None, None) == _lib.POLYPIC_EINVAL
    assert lib.polypic_mac_p2g(ctypes.byref(g), -1, 4, FAKE, None, 1.0, FAKE, None, FAKE, FAKE,
                               0, None, None) == _lib.POLYPIC_EINVAL
    assert lib.polypic_mac_p2g(ctypes.byref(grid(2, 36, 36)), 10, 4, FAKE, None, 1.0, FAKE, None,
                               FAKE, FAKE, 0, None, None) == _lib.POLYPIC_EINVAL
    # grid update: null arrays, negative bc_layers, null gravity
    assert lib.polypic_mac_grid_update(ctypes.byref(g), 1e-4, g3, 1, None, FAKE, FAKE,
                                       None) == _lib.POLYPIC_EINVAL
    assert lib.polypic_mac_grid_update(ctypes.byref(g), 1e-4, g3, -1, FAKE, FAKE, FAKE,
                                       None) == _lib.POLYPIC_EINVAL
    assert lib.polypic_mac_grid_update(ctypes.byref(g), 1e-4, None, 1, FAKE, FAKE, FAKE,
                                       None) == _lib.POLYPIC_EINVAL
    # G2P: unpaired F / mass, null output, bad mode count; P = 0 is a no-op
    assert lib.polypic_mac_g2p(ctypes.byref(g), 10, 4, 1e-4, FAKE, FAKE, None, None, FAKE, FAKE,
                               None, None, None, None, None) == _lib.POLYPIC_EINVAL
    assert lib.polypic_mac_g2p(ctypes.byref(g), 10, 4, 1e-4, FAKE, FAKE, None, None, FAKE, None,
                               None, FAKE, None, None, None) == _lib.POLYPIC_EINVAL
    assert lib.polypic_mac_g2p(ctypes.byref(g), 10, 4, 1e-4, FAKE, FAKE, None, None, None, None,
                               None, None, None, None, None) == _lib.POLYPIC_EINVAL
    assert lib.polypic_mac_g2p(ctypes.byref(g), 10, 9, 1e-4, FAKE, FAKE, None, None, FAKE, None,
                               None, None, None, None, None) == _lib.POLYPIC_EINVAL
    assert lib.polypic_mac_g2p(ctypes.byref(g), 0, 4, 1e-4, None, None, None, None, None, None,
                               None, None, None, None, None) == _lib.POLYPIC_OK


def test_mixture_and_affine_calls_reject_bad_arguments_on_the_host():
    lib = _lib.load()
    g = grid()
    g3 = (ctypes.c_float * 3)(0.0, -9.8, 0.0)
    # mixture P2G: phase and mass_f are required for P > 0
    assert lib.polypic_mixture_p2g(ctypes.byref(g), 10, 4, FAKE, None, FAKE, None, FAKE, None,
                                   FAKE, FAKE, 0, None, None) == _lib.POLYPIC_EINVAL
    assert lib.polypic_mixture_p2g(ctypes.byref(g), 10, 4, FAKE, FAKE, None, None, FAKE, None,
                                   FAKE, FAKE, 0, None, None) == _lib.POLYPIC_EINVAL
    assert lib.polypic_mixture_p2g(ctypes.byref(g), 10, 3, FAKE, FAKE, FAKE, None, FAKE, None,
                                   FAKE, FAKE, 0, None, None) == _lib.POLYPIC_EINVAL
    assert lib.polypic_mixture_grid_update(ctypes.byref(g), 1e-4, g3, -1, FAKE, FAKE, FAKE,
                                           None) == _lib.POLYPIC_EINVAL
    # mixture G2P: phase_in required, unpaired per-particle arrays rejected
    assert lib.polypic_mixture_g2p(ctypes.byref(g), 10, 4, 1e-4, FAKE, FAKE, None, None, None,
                                   FAKE, None, None, None, None, None, None, None, None,
                                   None) == _lib.POLYPIC_EINVAL
    assert lib.polypic_mixture_g2p(ctypes.byref(g), 10, 4, 1e-4, FAKE, FAKE, FAKE, None, None,
                                   FAKE, None, None, None, FAKE, None, None, None, None,
                                   None) == _lib.POLYPIC_EINVAL
    # affine P2G: bad dt, bad mode count, null outputs
    assert lib.polypic_p2g_affine(ctypes.byref(g), 10, 4, float("nan"), FAKE, None, None, 1.0,
                                  FAKE, None, FAKE, FAKE, 0, None, None) == _lib.POLYPIC_EINVAL
    assert lib.polypic_p2g_affine(ctypes.byref(g), 10, 2, 1e-4, FAKE, None, None, 1.0, FAKE,
                                  None, FAKE, FAKE, 0, None, None) == _lib.POLYPIC_EINVAL
    assert lib.polypic_p2g_affine(ctypes.byref(g), 10, 4, 1e-4, FAKE, None, None, 1.0, FAKE,
                                  None, None, FAKE, 0, None, None) == _lib.POLYPIC_EINVAL
