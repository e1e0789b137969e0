"""PolyPIC particle/grid transfers for AMD Instinct MI355X (gfx950).

Hand-written HIP kernels behind the C ABI of include/polypic.h
(libpolypic.so), with a thin torch binding:

* ``ops``      -- one Python function per C entry point (same names);
* ``stepper``  -- ``ParticleSet``: buffers of one particle set and its grid,
                  stepped by sort -> P2G -> grid update -> G2P.

Importing the package loads libpolypic.so and fails if it has not been built.
"""
from ._lib import LIB_PATH, PolyPICError, load, polypic_grid

load()  # fail loudly here if the HIP library is missing

from . import ops  # noqa: E402
from .ops import (  # noqa: E402
    polypic_autotune_p2g,
    polypic_get_p2g_config,
    polypic_set_p2g_config,
    grid_from_spec,
    make_grid,
    polypic_g2p,
    polypic_grid_update,
    polypic_p2g,
    polypic_sort,
    polypic_sort_workspace_bytes,
)
from .stepper import ParticleSet  # noqa: E402
from .autograd import PolyPICSteps, polypic_steps  # noqa: E402

__all__ = [
    "LIB_PATH", "PolyPICError", "polypic_grid", "ops", "make_grid", "grid_from_spec",
    "polypic_sort", "polypic_sort_workspace_bytes", "polypic_p2g", "polypic_grid_update",
    "polypic_g2p", "polypic_autotune_p2g", "polypic_get_p2g_config", "polypic_set_p2g_config",
    "ParticleSet", "PolyPICSteps", "polypic_steps",
]
