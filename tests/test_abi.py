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


@pytest.mark.parametrize("n_modes", [0, 2, 5, 9, 26, 28])
def test_p2g_rejects_bad_mode_count(n_modes):
    lib = _lib.load()
    g = grid()
    st = lib.polypic_p2g(ctypes.byref(g), 10, n_modes, FAKE, None, 1.0, FAKE, None, FAKE, FAKE,
                         0, None, None)
    assert st == _lib.POLYPIC_EINVAL


def test_p2g_rejects_null_and_bad_sizes():
    lib = _lib.load()
    g = grid()
    assert lib.polypic_p2g(ctypes.byref(g), 10, 4, None, None, 1.0, FAKE, None, FAKE, FAKE, 0,
                           None, None) == 1
    assert lib.polypic_p2g(ctypes.byref(g), 10, 4, FAKE, None, 1.0, FAKE, None, None, FAKE, 0,
                           None, None) == 1
    assert lib.polypic_p2g(ctypes.byref(g), -5, 4, FAKE, None, 1.0, FAKE, None, FAKE, FAKE, 0,
                           None, None) == 1
    assert lib.polypic_p2g(ctypes.byref(g), 1 << 31, 4, FAKE, None, 1.0, FAKE, None, FAKE, FAKE,
                           0, None, None) == 1
    bad = grid(2, 36, 36)
    assert lib.polypic_p2g(ctypes.byref(bad), 10, 4, FAKE, None, 1.0, FAKE, None, FAKE, FAKE, 0,
                           None, None) == 1
    neg = grid(dx=-1.0)
    assert lib.polypic_p2g(ctypes.byref(neg), 10, 4, FAKE, None, 1.0, FAKE, None, FAKE, FAKE, 0,
                           None, None) == 1
    assert lib.polypic_p2g(ctypes.byref(g), 10, 4, FAKE, None, float("nan"), FAKE, None, FAKE,
                           FAKE, 0, None, None) == 1


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
    assert lib.polypic_sort(ctypes.byref(g), 100, FAKE, FAKE, FAKE, FAKE, 16, None, None) == 4
    assert lib.polypic_sort(ctypes.byref(g), 100, None, FAKE, FAKE, FAKE, 1 << 20, None,
                            None) == 1
    assert lib.polypic_sort(ctypes.byref(g), 0, None, None, None, None, 0, None, None) == 0
