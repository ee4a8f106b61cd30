"""Seeded synthetic inputs shared by the CPU oracle, the GPU tests and the benchmark.

This module only draws random numbers and arranges them into arrays.  It holds
none of the method's arithmetic (no tensor, no contraction, no solver): the
response ``y = X w + sigma * eps`` is the data model of the synthetic
experiments (Section 5.4, "Comparing on synthetic data"), not part of the
regression method.

Every workload is a pure function of its seed.  Random numbers that the method
itself would draw (the Nystrom landmark indices of Section 6.1) are drawn here
and handed to both sides as inputs.
"""
from .generators import (  # noqa: F401
    CONFIGS,
    Workload,
    lambda_grid,
    landmark_draws,
    make_workload,
    planted_classification,
    planted_regression,
    random_alpha,
    random_symmetric_packed_values,
)
