"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package only generates data: element vertices, slip directions,
friction parameters and random slip-rate vectors.  It holds none of the
method's arithmetic (no Green's functions, no cluster tree, no low-rank
approximation, no products), so that the oracle and the GPU path stay
independent while reading identical input bits.
"""
from .faults import (  # noqa: F401
    PlanarRectFault,
    planar_rect_fault,
    config_fault,
    loguniform_rates,
    friction_params,
    ensemble_params,
    WORKLOADS,
    SIZE_SWEEP,
    LATTICE_SWEEP,
    TriangleFault,
    curved_thrust_fault,
    config_triangle_fault,
    TRIANGLE_WORKLOADS,
    triangle_friction_params,
)
