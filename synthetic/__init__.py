"""Seeded synthetic workload inputs shared by the test oracle and the HIP path.

This package holds only workload parameters and seeded random draws (noise
vectors, probe blocks, observation locations). It contains none of the
assimilation arithmetic: no model integration, no covariance square root, no
linear algebra. Each side (the CPU oracle and the GPU library) turns these
draws into a concrete problem with its own code.
"""

from .draws import (  # noqa: F401
    L96Workload,
    WORKLOADS,
    workload,
    obs_locations,
    l96_draws,
    probe_block,
    batch_workloads,
    BATCH_N_VALUES,
    advdiff_draws,
    ADV_GRIDS,
    CYCLED,
    cycled_draws,
    net_init,
)
