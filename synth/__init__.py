"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This package holds no arithmetic of the homogenization method itself: it only
draws microstructures (phase indicator grids, conductivity fields) and builds
material tables.  Both the CPU oracle and the HIP library receive the arrays
produced here as plain inputs.
"""
from .microstructure import (  # noqa: F401
    isotropic_mandel, isotropic_conductivity, spheres, circles2d, laminate,
    gaussian_random_field, conductivity_grf, workload, batch_workload, batch_workload_parallel,
)
