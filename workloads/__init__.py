"""Seeded synthetic inputs for the additive sweeping preconditioner.

This module only generates data: velocity fields c(x) on the interior grid
and right-hand sides f(x).  It holds none of the method's arithmetic (no PML,
no operator, no solver) so that the CPU oracle and the GPU path can consume
identical inputs without sharing any code of the method.

Grid convention (Section 3.1, column-major ordering): points x = (i1*h, ..., id*h)
with 1 <= ik <= n and h = 1/(n+1); arrays are returned with shape (n,)*d indexed
[i1-1, i2-1, ...] and are flattened with order="F" (i1 fastest) by ``flat``.
"""
from .fields import (  # noqa: F401
    grid_coords,
    flat,
    velocity_constant,
    velocity_lens2d,
    velocity_lens3d,
    velocity_random,
    velocity_waveguide2d,
    variation_widths,
    gaussian_source,
    wave_packet,
    paper_workload,
    paper_workload3d,
    PAPER_FIELDS,
    PAPER_SIZES,
    PAPER_SIZES_3D,
    seeded_centres,
    workload,
    WORKLOADS,
)
from .serving import request_stream, materialize, velocity_of, sources_of  # noqa: F401
