"""Pins of the oracle's octree (Section 4) on hand-built inputs.

Refinement rule (integer-exact reading of the subblock overlap estimate):
count(node) = sum_sb floor(ntets(sb) * |bbox(sb) cap node| / |bbox(sb)|),
refine iff count > threshold and level < max_level.
"""

import numpy as np

from synth import lattice_positions, zeldovich_positions


def _squeezed(np_=8, frac=0.5):
    """Lattice compressed into [0, frac)^3: everything in the first octant."""
    pos = lattice_positions(np_).astype(np.float64) * frac
    return pos.astype(np.float32)


def test_refines_only_where_the_tets_are(orc):
    pos = _squeezed()
    nodes = orc.build_octree(pos, block=2, max_level=2, subblock=2, threshold=1000)
    assert nodes["count"][0] == 6 * 8 ** 3
    lv = nodes["level"]
    assert list(np.bincount(lv)) == [1, 8, 8]
    assert nodes["first_child"][0] == 1
    # only octant (0,0,0) of level 1 is refined, and it is the first in Morton order
    l1 = nodes[lv == 1]
    assert l1["first_child"][0] == 9 and np.all(l1["first_child"][1:] == -1)
    assert l1["count"][0] == 6 * 8 ** 3 and np.all(l1["count"][1:] == 0)
    assert (nodes["leaf_id"] >= 0).sum() == 15
    assert list(nodes["leaf_id"][nodes["leaf_id"] >= 0]) == list(range(15))


def test_count_equal_to_threshold_does_not_refine(orc):
    pos = _squeezed()
    total = 6 * 8 ** 3
    nodes = orc.build_octree(pos, block=2, max_level=2, subblock=2, threshold=total)
    assert len(nodes) == 1 and nodes["leaf_id"][0] == 0
    nodes = orc.build_octree(pos, block=2, max_level=2, subblock=2, threshold=total - 1)
    assert len(nodes) > 1


def test_complete_tree_when_every_count_exceeds(orc):
    pos = zeldovich_positions(8, 0.3, seed=31)
    nodes = orc.build_octree(pos, block=2, max_level=2, subblock=4, threshold=0)
    assert list(np.bincount(nodes["level"])) == [1, 8, 64]
    # Morton order within a level, x most significant
    l2 = nodes[nodes["level"] == 2]
    keys = []
    for n in l2:
        k = 0
        for b in (1, 0):
            k = (k << 3) | (((n["ix"] >> b) & 1) << 2) | (((n["iy"] >> b) & 1) << 1) | ((n["iz"] >> b) & 1)
        keys.append(k)
    assert keys == sorted(keys) and len(set(keys)) == 64
    # counts are additive estimates: children never exceed a parent's subblocks' total
    assert nodes["count"][0] == 6 * 8 ** 3


def test_complete_tree_deposit_equals_uniform_grid(orc):
    pos = zeldovich_positions(8, 0.6, seed=32)
    B = 4
    nodes = orc.build_octree(pos, block=B, max_level=1, subblock=4, threshold=0)
    leaves = nodes[nodes["leaf_id"] >= 0]
    assert len(leaves) == 8
    out, _ = orc.deposit_octree(pos, nodes, np.arange(8), block=B)
    uni, _ = orc.deposit_uniform(pos, 2 * B)
    for s, lf in enumerate(leaves):
        blk = uni[lf["ix"] * B:(lf["ix"] + 1) * B, lf["iy"] * B:(lf["iy"] + 1) * B,
                  lf["iz"] * B:(lf["iz"] + 1) * B]
        assert np.max(np.abs(out[s] - blk)) <= 1e-15


def test_coarse_leaf_is_block_sum_of_fine_grid(orc):
    pos = _squeezed(8, 0.5)
    B = 2
    nodes = orc.build_octree(pos, block=B, max_level=2, subblock=2, threshold=1000)
    leaves = nodes[nodes["leaf_id"] >= 0]
    out, _ = orc.deposit_octree(pos, nodes, np.arange(len(leaves)), block=B)
    fine, _ = orc.deposit_uniform(pos, B * 4)
    assert abs(out.sum() - 1.0) <= 1e-12
    for s, lf in enumerate(leaves):
        f = 1 << (2 - lf["level"])          # fine cells per leaf cell, per axis
        blk = fine[lf["ix"] * B * f:(lf["ix"] + 1) * B * f, lf["iy"] * B * f:(lf["iy"] + 1) * B * f,
                   lf["iz"] * B * f:(lf["iz"] + 1) * B * f]
        coarse = blk.reshape(B, f, B, f, B, f).sum(axis=(1, 3, 5))
        assert np.max(np.abs(out[s] - coarse)) <= 1e-14


def test_count_is_floor_of_overlap_share(orc):
    """Hand-computed counts: one subblock of 4^3 cubes (384 tets), bbox [0,3)^3 on G=8.

    Particles at i*0.1 per axis -> finest units i*0.8 in [0, 2.4], snapped outward
    to [0,3) (volume 27).  Level-2 nodes have side 2, so the first octant's
    children overlap the bbox by 8, 4, 2 or 1 lattice volumes:
    floor(384*8/27)=113, floor(384*4/27)=56, floor(384*2/27)=28, floor(384/27)=14.
    """
    pos = (lattice_positions(4).astype(np.float64) * 0.4).astype(np.float32)
    nodes = orc.build_octree(pos, block=2, max_level=2, subblock=4, threshold=100)
    assert nodes["count"][0] == 384
    l2 = nodes[nodes["level"] == 2]
    assert len(l2) == 8
    want = {0: 113, 1: 56, 2: 28, 3: 14}
    for n in l2:
        k = int(n["ix"] + n["iy"] + n["iz"])
        assert n["count"] == want[k], (n, want[k])
