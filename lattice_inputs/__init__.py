"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package generates inputs only: gauge fields, random SU(3) matrices,
random spinors and the workload recipes.  It holds none of the arithmetic of
the method itself (no Dirac operator, no solver, no contraction), so the CPU
oracle and the GPU library can both be fed from it without sharing code.
"""

from .gauge import make_gauge, unit_gauge, random_su3, random_spinor, lattice_volume
from .workloads import WORKLOADS, Workload, get_workload

__all__ = [
    "make_gauge",
    "unit_gauge",
    "random_su3",
    "random_spinor",
    "lattice_volume",
    "WORKLOADS",
    "Workload",
    "get_workload",
]
