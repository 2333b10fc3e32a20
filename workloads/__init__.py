"""Seeded synthetic workloads for the IETI-DP magnetostatics solver.

This package only *describes* problems: patch grids, geometry parameters,
spline degree and refinement, the patch-to-subdomain partition, per-patch
reluctivity and the source current density J (as a vectorised callable).
It holds none of the solver's arithmetic (no basis functions, no assembly,
no tree, no linear algebra), so both the CPU oracle and the GPU library can
consume the same inputs without sharing any method code.
"""
from .problem import Problem, patch_index, patch_coords
from .configs import make_config, config_names
from .partition import greedy_partition, partition_is_admissible

__all__ = [
    "Problem",
    "patch_index",
    "patch_coords",
    "make_config",
    "config_names",
    "greedy_partition",
    "partition_is_admissible",
]
