"""Snapshot ingest and coarse octree levels, written out from their definitions.

TEST INFRASTRUCTURE ONLY (the test suite and the benchmark's CPU-baseline leg
are the only users; nothing here touches the GPU library).

- Ingest (Section 3): tracers arrive in any order with unique IDs that give
  their Lagrangian position; sorted by ID they form the Lagrangian grid.
  Record r belongs at slot ids[r] - id_base, slot (i*np1 + j)*np2 + k holding
  particle (i, j, k).
- Coarse levels (Section 8, future work): a node at level l of the octree
  covers box/2^l per axis; its coarse representation is the cell mass of the
  tessellation on the node's B^3 cells of side box/(B 2^l), i.e. the
  cell-averaged Eq. (1) at that resolution, computed here directly by the
  oracle's depositor on the node's region.
"""

from __future__ import annotations

import numpy as np

from .oracle import deposit_uniform


def reorder_by_id(ids, pos_in, np_, id_base: int = 0):
    """(grid float32 [np0, np1, np2, 3] with unnamed slots NaN, named-once mask [np0*np1*np2],
    (out of range, duplicates, missing)).  Slots named by several records are NaN here: the
    result there is any one of them."""
    g = tuple(int(x) for x in np_)
    n_slots = g[0] * g[1] * g[2]
    ids = np.asarray(ids, dtype=np.int64)
    pos_in = np.asarray(pos_in, dtype=np.float32).reshape(-1, 3)
    out = np.full((n_slots, 3), np.nan, dtype=np.float32)
    times = np.zeros(n_slots, dtype=np.int64)
    bad = 0
    for r in range(ids.size):
        slot = int(ids[r]) - int(id_base)
        if slot < 0 or slot >= n_slots:
            bad += 1
            continue
        times[slot] += 1
        out[slot] = pos_in[r]
    dup = int(np.maximum(times - 1, 0).sum())
    missing = int((times == 0).sum())
    out[times > 1] = np.nan
    return out.reshape(g + (3,)), times == 1, (bad, dup, missing)


def coarse_levels(pos, nodes, block: int, box: float = 1.0, mass: float = 1.0,
                  density: bool = False, nthreads: int = 0) -> np.ndarray:
    """Every node's B^3 cell masses (or densities) at its own resolution: float64
    [len(nodes), B, B, B] in node order."""
    B = int(block)
    out = np.zeros((len(nodes), B, B, B), dtype=np.float64)
    for n, nd in enumerate(nodes):
        level = int(nd["level"])
        nc = B << level
        lo = (B * int(nd["ix"]), B * int(nd["iy"]), B * int(nd["iz"]))
        m, _ = deposit_uniform(pos, nc, box=box, mass=mass, region=(lo, (B, B, B)),
                               nthreads=nthreads)
        if density:
            m = m * (nc / box) ** 3
        out[n] = m
    return out
