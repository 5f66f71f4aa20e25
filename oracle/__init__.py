"""FP64 CPU oracle for phase-space-element density deposition.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only users.  The GPU library never imports, links or
calls anything here, and this package imports nothing from it.
"""

from .oracle import (  # noqa: F401
    build_oracle,
    lib,
    Counters,
    clip_tet_box,
    clip_tet_box_paper,
    cube_tets,
    deposit_uniform,
    build_octree,
    deposit_octree,
    NODE_DTYPE,
    surrogate_examples,
    TRIVIAL,
    PAPER,
)
from .ingest import reorder_by_id, coarse_levels  # noqa: F401
