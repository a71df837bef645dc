"""Seeded synthetic inputs for the short-range particle-particle force.

This package is shared by the oracle-based tests, the GPU parity tests and
the benchmark.  It only draws particle positions, masses, cotangent vectors
and the polynomial grid-force coefficients; it evaluates no part of the
short-range force itself.
"""
from .configs import (Workload, make_config, config_names, uniform_gauss,
                      plummer_clustered, nfw_clustered, add_ghost_shell,
                      cotangent)
from .fgrid import fit_fgrid, FGridFit

__all__ = ["Workload", "make_config", "config_names", "uniform_gauss",
           "plummer_clustered", "nfw_clustered", "add_ghost_shell",
           "cotangent", "fit_fgrid", "FGridFit"]
