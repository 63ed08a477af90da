"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle tests.

This package draws point clouds and initial fields only. It holds none of the
method's arithmetic (no equilibrium, no interpolation, no collision), so that
the oracle and the GPU path can both consume its output without sharing code.
"""
from .clouds import (  # noqa: F401
    Cloud,
    jittered_lattice,
    annulus_poisson,
    batched_tgv_specs,
    tgv_initial_velocity,
    random_field,
)
