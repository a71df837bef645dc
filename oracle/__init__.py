"""Float64 CPU oracle for the short-range particle-particle force.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline call this package; the GPU library never does, and this package
never imports the GPU library.  It shares no code with the HIP path.

* ``force`` / ``force_vjp``: the C cell-list oracle (``sr_oracle.c``),
  float64, OpenMP over targets.
* ``brute``: an independent NumPy all-pairs implementation for tiny inputs.
* ``rollout``: the stream-kick-stream subcycle map and its adjoint in float64.
* ``binning``: the chaining-mesh cell list (keys, stable order, records).
"""
from .clib import (force, force_vjp, num_threads, build, library_path,
                   rel_err_floored)
from . import brute, rollout, binning

__all__ = ["force", "force_vjp", "num_threads", "build", "library_path",
           "rel_err_floored", "brute", "rollout", "binning"]
