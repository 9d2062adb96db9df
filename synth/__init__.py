"""Seeded synthetic inputs shared by the tests, the oracle checks and the benchmark.

This package generates *inputs only*: quenched U(1) gauge fields, right-hand sides
and the random vectors that the adaptive multigrid setup starts from.  It holds none
of the solver's arithmetic (no Dirac operator, no multigrid), so the GPU library and
the CPU oracle can both consume its outputs without sharing any method code.
"""

from .gauge import (metropolis_u1, metropolis_u1_device, plaquette_angles, mean_plaquette, topological_charge,
                    links_from_angles)
from .vectors import gaussian, gaussian_device, z2_noise, point_source, setup_randoms, level_shapes

__all__ = [
    "metropolis_u1",
    "metropolis_u1_device",
    "plaquette_angles",
    "mean_plaquette",
    "topological_charge",
    "links_from_angles",
    "gaussian",
    "gaussian_device",
    "z2_noise",
    "point_source",
    "setup_randoms",
    "level_shapes",
]
