"""GPU octree (Section 4) against the oracle.

Node arrays must be bit-identical (the count rule is integer-exact); leaf
cell masses within 1e-5 relative L1 (FP32 output) of the oracle's.
"""

import functools

import numpy as np
import pytest
import torch

from synth import apply_clumps, lattice_positions, zeldovich_positions

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def psd():
    import os
    import paper_1612_09491_amd as psd
    if not os.path.exists(psd.LIB_PATH):
        from paper_1612_09491_amd import build
        build.build()
    return psd


def _dev(pos):
    return torch.from_numpy(np.ascontiguousarray(pos)).to(torch.device("cuda:0"))


def _same_nodes(got, ref):
    assert len(got) == len(ref)
    for f in ("level", "ix", "iy", "iz", "first_child", "leaf_id", "count"):
        assert np.array_equal(got[f], ref[f]), f


CASES = [
    # (name, positions, block, max_level, subblock, threshold)
    ("squeezed", lambda: (lattice_positions(8).astype(np.float64) * 0.5).astype(np.float32), 2, 2, 2, 1000),
    ("floor_counts", lambda: (lattice_positions(4).astype(np.float64) * 0.4).astype(np.float32), 2, 2, 4, 100),
    ("complete", lambda: zeldovich_positions(8, 0.3, seed=31), 2, 2, 4, 0),
    ("zel32_adaptive", lambda: zeldovich_positions(32, 1.5, seed=61), 4, 3, 8, 3000),
    ("clumps64", lambda: apply_clumps(zeldovich_positions(64, 2.0, seed=62), seed=63), 4, 4, 8, 20000),
    # leaves of 3^3 cells (a block that is not a power of two) at levels 2 and 3
    ("zel32_block3", lambda: zeldovich_positions(32, 1.5, seed=64), 3, 3, 8, 3000),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_tree_bit_exact(psd, orc, case):
    name, mk, B, L, S, T = case
    pos = mk()
    ref = orc.build_octree(pos, block=B, max_level=L, subblock=S, threshold=T)
    tree = psd.build_octree(_dev(pos), block=B, max_level=L, subblock=S, threshold=T)
    got = tree.to_numpy()
    _same_nodes(got, ref)
    assert tree.n_leaves == int((ref["leaf_id"] >= 0).sum())


def test_capacity_error_reports_size(psd, orc):
    pos = zeldovich_positions(8, 0.3, seed=31)
    with pytest.raises(psd.PsdError) as e:
        psd.build_octree(_dev(pos), block=2, max_level=2, subblock=4, threshold=0, capacity=10)
    assert e.value.code == psd.PSD_ERR_CAPACITY and e.value.n_nodes == 73


@pytest.mark.parametrize("case", CASES[1:], ids=[c[0] for c in CASES[1:]])
def test_leaf_deposit_matches_oracle(psd, orc, case):
    name, mk, B, L, S, T = case
    pos = mk()
    ref_nodes = orc.build_octree(pos, block=B, max_level=L, subblock=S, threshold=T)
    nl = int((ref_nodes["leaf_id"] >= 0).sum())
    ref, _ = orc.deposit_octree(pos, ref_nodes, np.arange(nl), block=B)
    pt = _dev(pos)
    tree = psd.build_octree(pt, block=B, max_level=L, subblock=S, threshold=T)
    ms = torch.zeros(1, dtype=torch.float64, device=pt.device)
    out = psd.deposit_octree(pt, tree, mass_sum=ms)
    dens = psd.deposit_octree(pt, tree, flags=psd.PSD_OUT_DENSITY)
    torch.cuda.synchronize()
    got = out.double().cpu().numpy()
    l1 = np.abs(got - ref).sum() / np.abs(ref).sum()
    assert l1 <= 1e-5, l1
    assert abs(float(ms.item()) - 1.0) <= 1e-9
    # density = mass / h^3 with h = 1 / (B 2^level) of each leaf
    levels = ref_nodes["level"][ref_nodes["leaf_id"] >= 0]
    h3 = (1.0 / (B * 2.0 ** levels)) ** 3
    assert np.allclose(dens.double().cpu().numpy() * h3[:, None, None, None], got, rtol=2e-5,
                       atol=1e-12)


@pytest.mark.parametrize("tuning", [(960, 12, 1), (512, 4, 0), (2048, 7, 0), (1408, 12, 0),
                                    (1024, 12, 0)])
def test_leaf_deposit_launch_shapes_agree(psd, orc, tuning):
    """Cost order (no skipping of leafless levels) and other LDS buffers give the same
    leaves; the tree here has leaves at several levels and leafless ones above them."""
    name, mk, B, L, S, T = next(c for c in CASES if c[0] == "zel32_adaptive")
    pos = mk()
    pt = _dev(pos)
    tree = psd.build_octree(pt, block=B, max_level=L, subblock=S, threshold=T)
    base = psd.deposit_octree(pt, tree).double().cpu().numpy()
    got = psd.deposit_octree(pt, tree, tuning=tuning).double().cpu().numpy()
    assert np.abs(got - base).sum() / np.abs(base).sum() <= 1e-6


@functools.lru_cache(maxsize=1)
def _clump512():
    from synth import workload
    return workload("clump512_octree")


def test_clump512_tree_and_sampled_leaves(psd, orc):
    """Full size: 512^3 particles + clumps, B=16, 4 levels, threshold 2^20."""
    pos, p = _clump512()
    B, L, T = p["block"], p["max_level"], p["threshold"]
    ref = orc.build_octree(pos, block=B, max_level=L, subblock=8, threshold=T)
    pt = _dev(pos)
    tree = psd.build_octree(pt, block=B, max_level=L, subblock=8, threshold=T)
    _same_nodes(tree.to_numpy(), ref)
    print("levels:", np.bincount(ref["level"][ref["leaf_id"] >= 0]))
    ms = torch.zeros(1, dtype=torch.float64, device=pt.device)
    out = psd.deposit_octree(pt, tree, mass_sum=ms)
    torch.cuda.synchronize()
    assert abs(float(ms.item()) - 1.0) <= 1e-9
    got = out.double().cpu().numpy()
    assert abs(got.sum() - 1.0) <= 1e-4
    rng = np.random.default_rng(3)
    sel = np.sort(rng.choice(tree.n_leaves, size=2, replace=False))
    want, _ = orc.deposit_octree(pos, ref, sel, block=B)
    l1 = np.abs(got[sel] - want).sum() / np.abs(want).sum()
    print(f"sampled leaves {sel.tolist()}: L1 {l1:.3e}")
    assert l1 <= 1e-5


def test_adaptive_tree_at_scale(psd, orc):
    """128^3 particles (12.6M tetrahedra) squeezed toward a corner (x -> x^2 per axis over
    a Zel'dovich grid): with threshold 1e5 the tree has leaves at levels 2, 3 and 4.  The
    node array is bit-identical to the oracle's; three leaves of every level match the
    oracle within the FP32 bar; the root's coarse block (internal-node sums) matches the
    oracle's direct 16^3 deposit."""
    base = zeldovich_positions(128, 0.5, seed=91).astype(np.float64)
    pos = (base ** 2).astype(np.float32)
    kw = dict(block=16, max_level=4, subblock=8, threshold=100000)
    ref_nodes = orc.build_octree(pos, **kw)
    pt = _dev(pos)
    tree = psd.build_octree(pt, **kw)
    got_nodes = tree.to_numpy()
    _same_nodes(got_nodes, ref_nodes)
    leaf_nodes = np.nonzero(ref_nodes["leaf_id"] >= 0)[0]
    levels = ref_nodes["level"][leaf_nodes]
    assert set(np.unique(levels).tolist()) == {2, 3, 4}
    ms = torch.zeros(1, dtype=torch.float64, device=pt.device)
    out = psd.deposit_octree(pt, tree, mass_sum=ms)
    torch.cuda.synchronize()
    assert abs(float(ms.item()) - 1.0) <= 1e-9
    got = out.double().cpu().numpy()
    for lvl in (2, 3, 4):
        sel = leaf_nodes[levels == lvl]
        ids = ref_nodes["leaf_id"][sel[[0, len(sel) // 2, -1]]]
        ref, _ = orc.deposit_octree(pos, ref_nodes, ids, block=16)
        g = got[ids]
        l1 = np.abs(g - ref).sum() / np.abs(ref).sum()
        linf = np.abs(g - ref).max() / np.abs(ref).max()
        print(f"level {lvl} leaves {ids.tolist()}: L1 {l1:.3e} Linf {linf:.3e}", flush=True)
        assert l1 <= 1e-5 and linf <= 1e-5
    coarse = psd.octree_coarsen(tree, out).double().cpu().numpy()
    root_ref, _ = orc.deposit_uniform(pos, 16)
    l1 = np.abs(coarse[0] - root_ref).sum() / np.abs(root_ref).sum()
    print(f"root coarse block: L1 {l1:.3e}", flush=True)
    assert l1 <= 1e-5
