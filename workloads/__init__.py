"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds no arithmetic of the method: it only names workload
parameters (laser, foil, grid, particle counts) and draws seeded random
test states.  Every derived quantity (cell size, time step, particle
weight, radiation-reaction coefficient) is computed separately by each
consumer from these raw parameters.
"""
from .configs import PRESETS, preset, periods_to_steps, PRESETS_2D, preset2d  # noqa: F401
from .gen import (random_push_inputs, random_particles, random_fields, poisson_stream,  # noqa: F401
                  random_particles2d, random_fields2d)
