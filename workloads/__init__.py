"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package holds no arithmetic of the method itself: it only builds mesh node
coordinates, physical parameters and seeded random perturbations.
"""
from .cases import (  # noqa: F401
    BC_WALL, BC_FARFIELD, BC_PERIODIC, GAUSS_HERMITE, NEWTON_COTES, BGK, SHAKHOV,
    FP64, FP32_MIXED, EXPLICIT, IMPLICIT, SWEEPS_AUTO, SWEEPS_LEVELS, SWEEPS_HYPERPLANES,
    uniform_nodes, tanh_nodes, cartesian_mesh, ogrid_mesh,
    couette, cavity, cavity_re, cylinder, periodic_box, shrink, case, CASE_NAMES,
    perturbation,
)
from .meshes import mesh_of, with_mesh, hybrid_square, hybrid_cavity, renumbered  # noqa: F401
