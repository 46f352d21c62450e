"""Seeded synthetic layer generators shared by the tests, the benchmark and the oracle checks.

This package holds input construction only: expansion-coefficient sets for homogeneous particulate
layers, their validity check, and the fixed workload shapes. It contains none of the radiative
transfer solver's arithmetic and imports neither the oracle nor the GPU binding.
"""

from .layers import (  # noqa: F401
    COEF_ROWS,
    LayerSet,
    hg_like_coefficients,
    differentiation_targets,
    positivity_ok,
    rayleigh_coefficients,
    workload,
    WORKLOADS,
)
