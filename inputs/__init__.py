"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module holds workload definitions and seeded input generators only:
geometry parameters, refractive-index tables, layer thicknesses, material
assignments and reflection probabilities.  It contains none of the method's
arithmetic (no ray tracing, no thin-film solve, no geometry derived from the
method) so that the oracle and the HIP path stay independent.
"""
from .workloads import (  # noqa: F401
    MAT_AIR, MAT_GLASS, MAT_SIO2, MAT_TIO2, MAT_AL2O3, MAT_AG, MAT_TA2O5, N_MAT,
    Workload, workload, WORKLOADS, make_inputs, small_variant,
)
