"""Correctness oracle for the PolyPIC transfer library -- TEST INFRASTRUCTURE ONLY.

* ``polypic_oracle``: plain FP64 numpy implementation of sort keys, P2G, grid
  update, G2P, advection and the F update (section 3 of the paper).
* ``exact``: an independent exact-rational brute force for tiny inputs.
* ``adjoint``: the FP64 reverse-mode gradient of a chain of steps.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The library does not depend on it in any way.
"""
