"""Seeded synthetic inputs shared by the GPU library's tests/benchmark and the oracle.

This package holds no arithmetic of the method (no equation of state, no
Maxwell construction, no collision): it only draws seeded random numbers and
shapes initial fields from densities, radii and positions that the caller
passes in.
"""
from .rng import splitmix64, uniform
from .fields import drop_indicator, two_drop_fields, lens_drops, collision_drops
from . import workloads

__all__ = ["splitmix64", "uniform", "drop_indicator", "two_drop_fields", "lens_drops",
           "collision_drops", "workloads"]
