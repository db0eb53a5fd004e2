"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only builds meshes, time grids and incident-pulse parameters.  It holds
none of the method's arithmetic (no basis functions, no quadrature, no kernels).
"""
from .meshes import icosphere, geodesic_sphere, torus, mesh_diameter
from .grids import equidistant_grid, graded_grid
from .configs import CONFIGS, get_config, pulse_direction

__all__ = ["icosphere", "geodesic_sphere", "torus", "mesh_diameter", "equidistant_grid", "graded_grid",
           "CONFIGS", "get_config", "pulse_direction"]
