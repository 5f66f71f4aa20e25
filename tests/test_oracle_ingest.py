"""Pins of the oracle's snapshot ingest (Section 3) and coarse octree levels (Section 8).

Ingest: a hand-worked example (golden file) with IDs out of range, a duplicate and
missing slots, and the round trip of a random permutation.  Coarse levels: additivity
of |T cap C| over the 2x2x2 children of a cell, checked against the oracle's fine
uniform grid summed in blocks, mass conservation at the root, and density = mass / h^3.
"""

import os

import numpy as np
import pytest

from synth import zeldovich_positions

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_ingest():
    sections, cur = {}, None
    for line in open(os.path.join(GOLDEN, "ingest_2x1x3.txt")):
        if line.startswith("#@"):
            cur = line[2:].split()[0]
            sections[cur] = []
        elif line.strip() and not line.startswith("#"):
            sections[cur].append([float(x) for x in line.split()])
    return sections


def test_ingest_worked_example(orc):
    g = _golden_ingest()
    rec = np.array(g["records"])
    grid, once, check = orc.reorder_by_id(rec[:, 0].astype(np.int64), rec[:, 1:], (2, 1, 3),
                                          id_base=1)
    assert check == tuple(int(x) for x in g["check"][0])
    flat = grid.reshape(-1, 3)
    named = {int(r[0]): r[1:] for r in g["grid"]}
    assert sorted(np.nonzero(once)[0].tolist()) == sorted(named)
    for slot, xyz in named.items():
        assert np.array_equal(flat[slot], np.float32(xyz))


def test_ingest_permutation_round_trip(orc):
    pos = zeldovich_positions(6, 0.8, seed=71)
    n = pos.shape[0] ** 3
    perm = np.random.default_rng(72).permutation(n)
    records = pos.reshape(-1, 3)[perm]
    grid, once, check = orc.reorder_by_id(perm + 5, records, pos.shape[:3], id_base=5)
    assert check == (0, 0, 0) and once.all()
    assert np.array_equal(grid, pos)


@pytest.fixture(scope="module")
def tree_case(orc):
    pos = zeldovich_positions(12, 0.7, seed=73)
    nodes = orc.build_octree(pos, block=4, max_level=2, subblock=4, threshold=1500)
    return pos, nodes


def test_coarse_levels_additive(orc, tree_case):
    """A node's coarse cells equal block sums of the finest uniform grid over its region."""
    pos, nodes = tree_case
    B, L = 4, 2
    assert (nodes["first_child"] >= 0).any(), "the case must have internal nodes"
    coarse = orc.coarse_levels(pos, nodes, B)
    fine, _ = orc.deposit_uniform(pos, B << L)
    for n, nd in enumerate(nodes):
        f = 1 << (L - int(nd["level"]))          # fine cells per coarse cell, per axis
        s = B * f
        x0, y0, z0 = (s * int(nd[k]) for k in ("ix", "iy", "iz"))
        blk = fine[x0:x0 + s, y0:y0 + s, z0:z0 + s].reshape(B, f, B, f, B, f).sum(axis=(1, 3, 5))
        assert np.allclose(coarse[n], blk, rtol=1e-12, atol=1e-15), n
    root = coarse[nodes["level"] == 0][0]
    assert abs(root.sum() - 1.0) <= 1e-12


def test_coarse_levels_density(orc, tree_case):
    pos, nodes = tree_case
    m = orc.coarse_levels(pos, nodes[:9], 4, box=1.0)
    d = orc.coarse_levels(pos, nodes[:9], 4, box=1.0, density=True)
    for n, nd in enumerate(nodes[:9]):
        h3 = (1.0 / (4 << int(nd["level"]))) ** 3
        assert np.allclose(d[n] * h3, m[n], rtol=1e-14, atol=0)
