"""Seeded synthetic inputs shared by the tests, the bench and the smoke check.

This package holds no arithmetic of the estimator: it only draws the problem
inputs (locations, integration limits, request streams, random lower-triangular
factors with a tile-low-rank structure). Both the HIP path and the oracle take
what it produces as plain arrays.
"""

from .workloads import (  # noqa: F401
    GOLDEN_GAMMA,
    splitmix64,
    uniform01,
    grid_xy,
    upper_limits_uniform,
    CONFIGS,
    config,
    random_tlr_factor,
    serving_stream,
)
