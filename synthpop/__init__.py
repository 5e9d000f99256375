"""Seeded synthetic inputs shared by the GPU path's tests/bench and the CPU oracle.

This package holds no arithmetic of the epidemic method itself: it only draws
populations (ages, households, occupations, workplaces, initial infections) and
holds the parameter sets of the workloads.  Both sides receive these arrays as
inputs; neither side's computation lives here.
"""
from .population import (Population, make_population, replicate_population,  # noqa: F401
                         extract_replicate, split_replicates)
from .configs import workload, WORKLOADS  # noqa: F401
