"""PolyPIC particle/grid transfers for AMD Instinct MI355X (gfx950).

Hand-written HIP kernels behind the C ABI of include/polypic.h
(libpolypic.so), with a thin torch binding:

* ``ops``      -- one Python function per C entry point (same names);
* ``stepper``  -- ``ParticleSet``: buffers of one particle set and its grid,
                  stepped by sort -> P2G -> grid update -> G2P;
* ``batch``    -- ``BatchedParticleSet``: many scenes stepped by one launch per
                  phase, capturable as a HIP graph;
* ``autograd`` -- ``PolyPICSteps``: differentiable steps (hand-written adjoint).

Importing the package loads libpolypic.so and fails if it has not been built.
"""
from ._lib import LIB_PATH, PolyPICError, load, polypic_grid

load()  # fail loudly here if the HIP library is missing

from . import ops  # noqa: E402
from ._lib import (  # noqa: E402
    POLYPIC_P2G_BRICKS,
    POLYPIC_P2G_CELLS,
    POLYPIC_P2G_DEFAULT,
    POLYPIC_SCHED_LINEAR,
    POLYPIC_SCHED_PERSISTENT,
    POLYPIC_SCHED_XCD,
)
from .ops import (  # noqa: E402
    Batch,
    P2GChoice,
    polypic_autotune_p2g,
    polypic_get_g2p_schedule,
    polypic_get_p2g_config,
    polypic_set_g2p_schedule,
    polypic_set_p2g_config,
    grid_from_spec,
    make_grid,
    polypic_g2p,
    polypic_g2p2g,
    polypic_grid_update,
    polypic_grid_update_clear,
    polypic_p2g,
    polypic_sort,
    polypic_sort_update,
    polypic_sort_update_workspace_bytes,
    polypic_sort_workspace_bytes,
)
from .stepper import (AffineParticleSet, MacParticleSet, MixtureParticleSet,  # noqa: E402
                      ParticleSet)
from .batch import BatchedParticleSet  # noqa: E402
from .autograd import PolyPICSteps, polypic_steps  # noqa: E402

__all__ = [
    "LIB_PATH", "PolyPICError", "polypic_grid", "ops", "make_grid", "grid_from_spec",
    "polypic_sort", "polypic_sort_workspace_bytes", "polypic_p2g", "polypic_grid_update",
    "polypic_grid_update_clear", "polypic_g2p", "polypic_g2p2g", "polypic_sort_update",
    "polypic_sort_update_workspace_bytes", "polypic_autotune_p2g", "polypic_get_p2g_config",
    "polypic_set_p2g_config", "polypic_get_g2p_schedule", "polypic_set_g2p_schedule",
    "P2GChoice", "Batch",
    "POLYPIC_P2G_BRICKS", "POLYPIC_P2G_CELLS", "POLYPIC_P2G_DEFAULT", "POLYPIC_SCHED_LINEAR",
    "POLYPIC_SCHED_PERSISTENT", "POLYPIC_SCHED_XCD",
    "ParticleSet", "MacParticleSet", "AffineParticleSet", "MixtureParticleSet",
    "BatchedParticleSet", "PolyPICSteps", "polypic_steps",
]
