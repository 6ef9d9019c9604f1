"""Seeded synthetic workloads shared by the oracle and the GPU path.

This package only draws random numbers and evaluates the workload recipe
(the Gaussian wells that make up the potential V(r), the grid shapes, the
window counts).  It holds none of the eigensolver, partitioning or transport
arithmetic: the oracle and the HIP library each compute those on their own.
"""
from .workloads import (Grid, Absorber, Workload, wells_potential, draw_wells,
                        workload, batch_workloads, CONFIGS)

__all__ = ["Grid", "Absorber", "Workload", "wells_potential", "draw_wells",
           "workload", "batch_workloads", "CONFIGS"]
