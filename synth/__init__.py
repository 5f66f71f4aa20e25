"""Seeded synthetic particle grids for the deposition tests and benchmark.

This package only draws inputs (particle positions on a Lagrangian grid); it
holds none of the deposition arithmetic.  Both the GPU path and the CPU
oracle consume its outputs, which is the only thing they share.
"""

from .zeldovich import (  # noqa: F401
    zeldovich_positions,
    apply_clumps,
    lattice_positions,
    jittered_lattice_positions,
    batched_box_specs,
    workload,
    WORKLOADS,
    TRAIN_SEED0,
    uniform_segments,
)
