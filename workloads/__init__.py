"""Seeded synthetic workloads: building prisms, sample points and time spans.

This package holds input generators only. It computes no shadow, no sun
position and no interval: both the CPU oracle and the HIP path consume
what it produces, and neither shares any other code.
"""
from .scenes import (  # noqa: F401
    Scene, Points, Span, Workload,
    make_c1, make_c2, make_c3, make_c4, make_c5,
    subset_points, concat_points, NYC,
)
