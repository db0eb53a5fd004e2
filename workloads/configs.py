"""The named workloads.

sphere320_eq10       320-triangle icosphere, 10 equidistant bases on [0,4], pulse along +z
sphere5120_graded64  5120-triangle icosphere, 64 graded bases on [0,8]
torus20480_graded128 20480-triangle torus (R=1, r=0.35), 128 graded bases on [0,10]
The small ones exist for tests whose CPU reference must finish in seconds.
"""
import numpy as np
from .meshes import icosphere, torus
from .grids import equidistant_grid, graded_grid


def pulse_direction(seed):
    """Unit vector: a normalised N(0, I_3) draw (PCG64, `seed`)."""
    d = np.random.default_rng(seed).standard_normal(3)
    return d / np.linalg.norm(d)


def _cfg(name, mesh, grid, d, width, t0, cutoff="bump"):
    return dict(name=name, mesh=mesh, grid=grid, direction=d, width=width, t0=t0, cutoff=cutoff)


CONFIGS = {
    "sphere320_eq10": lambda: _cfg("sphere320_eq10", icosphere(2), equidistant_grid(10, 4.0),
                                   np.array([0.0, 0.0, 1.0]), 0.25, 1.5),
    "sphere5120_graded64": lambda: _cfg("sphere5120_graded64", icosphere(4), graded_grid(64, 8.0, seed=2),
                                        pulse_direction(3), 0.15, 1.0 + 6 * 0.15),
    "torus20480_graded128": lambda: _cfg("torus20480_graded128", torus(128, 80), graded_grid(128, 10.0, seed=4),
                                         pulse_direction(5), 0.1, 1.35 + 6 * 0.1),
    # small cases for the oracle-backed tests
    "sphere80_eq6": lambda: _cfg("sphere80_eq6", icosphere(1), equidistant_grid(6, 3.0),
                                 np.array([0.0, 0.0, 1.0]), 0.3, 1.5),
    "sphere80_graded7": lambda: _cfg("sphere80_graded7", icosphere(1), graded_grid(7, 3.0, seed=11),
                                     pulse_direction(12), 0.3, 1.0 + 6 * 0.3),
    "torus64_graded6": lambda: _cfg("torus64_graded6", torus(8, 4), graded_grid(6, 3.0, seed=13),
                                    pulse_direction(14), 0.3, 1.35 + 6 * 0.3),
    "sphere20_eq5_erf": lambda: _cfg("sphere20_eq5_erf", icosphere(0), equidistant_grid(5, 3.0),
                                     np.array([0.0, 0.0, 1.0]), 0.3, 1.5, cutoff="erf"),
}


def get_config(name):
    return CONFIGS[name]()
