"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This package holds no arithmetic of the discretisation: it draws seeded
random vectors and evaluates closed-form flow fields at coordinates the
caller supplies.  Both the oracle side and the GPU side take their inputs
from here and from nowhere else.
"""
from .fields import (random_vector, taylor_green_2d, taylor_green_2d_unit,
                     tgv3d_velocity, tgv3d_pressure, kovasznay,
                     random_phase_velocity, nodal_velocity, nodal_scalar,
                     sine_vertex_map)

__all__ = ["random_vector", "taylor_green_2d", "taylor_green_2d_unit",
           "tgv3d_velocity", "tgv3d_pressure", "kovasznay",
           "random_phase_velocity", "nodal_velocity", "nodal_scalar",
           "sine_vertex_map"]
