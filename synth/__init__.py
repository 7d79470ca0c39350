"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle checks.

This package draws random numbers and nothing else: it holds none of the
method's arithmetic (no Tucker, no stitching, no tree logic).  Both the GPU
path and the CPU oracle are fed from here so that they see identical inputs.
"""

from .workloads import (  # noqa: F401
    Workload,
    WORKLOADS,
    get,
    series,
    queries,
    small_series,
)
