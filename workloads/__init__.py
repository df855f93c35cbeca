"""Seeded synthetic inputs for the HDMR / adaptive-sparse-grid workloads.

This package is the only code shared by the CPU oracle and the GPU path.  It
holds input generators (points, random surpluses, grid shapes of synthetic
models, the synthetic test function) and nothing of the approximation
method's arithmetic.
"""
from .synth import (  # noqa: F401
    CONFIGS,
    TestFunction,
    config,
    next_state_points,
    random_pairs,
    regular_levels,
    synthetic_regular_model,
    uniform_points,
)
