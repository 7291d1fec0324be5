"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This package only draws random matrices; it holds no part of the
product's arithmetic and imports neither ``oracle`` nor the HIP package.
"""
from .matrices import (CSC, BatchSpec, batch_instance, batch_packed, batch_spec, erdos_renyi, powerlaw_xmin,
                       protein_like, rmat, shuffle_within_columns, target_values, tie_heavy)
from .workloads import WORKLOADS, Workload, make_workload

__all__ = [
    "CSC", "BatchSpec", "batch_instance", "batch_packed", "batch_spec", "erdos_renyi", "powerlaw_xmin", "protein_like",
    "rmat", "shuffle_within_columns", "target_values", "tie_heavy", "WORKLOADS", "Workload", "make_workload",
]
