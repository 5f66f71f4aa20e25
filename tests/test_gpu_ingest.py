"""GPU parity of snapshot ingest (psd_reorder_by_id, Section 3) and coarse octree levels
(psd_octree_coarsen, Section 8) against the oracle.

Ingest is byte work: positions must match bit for bit, and the three check counts
exactly.  Coarse levels: each node's block against the oracle's direct deposit at the
node's resolution (relative L1 and Linf <= 1e-5, the FP32 grid tolerance), and against
the exact 2x2x2 block sums of the GPU's own leaves (each level rounds once to FP32:
<= 4e-7 per level of depth below the node).
"""

import functools
import os

import numpy as np
import pytest
import torch

from synth import workload, zeldovich_positions

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def psd():
    import paper_1612_09491_amd as psd
    if not os.path.exists(psd.LIB_PATH):
        from paper_1612_09491_amd import build
        build.build()
    return psd


def _dev():
    return torch.device("cuda:0")


def _ingest(psd, ids, rec, np_, id_base=0, fill=np.nan):
    dev = _dev()
    out = torch.full(tuple(np_) + (3,), fill, dtype=torch.float32, device=dev)
    chk = torch.full((3,), -7, dtype=torch.int64, device=dev)
    psd.reorder_by_id(torch.from_numpy(np.ascontiguousarray(ids, dtype=np.int64)).to(dev),
                      torch.from_numpy(np.ascontiguousarray(rec, dtype=np.float32)).to(dev),
                      np_, id_base=id_base, out=out, check=chk)
    torch.cuda.synchronize()
    return out.cpu().numpy(), tuple(int(x) for x in chk.cpu().numpy())


def test_ingest_worked_example(psd, orc):
    sections, cur = {}, None
    for line in open(os.path.join(GOLDEN, "ingest_2x1x3.txt")):
        if line.startswith("#@"):
            cur = line[2:].split()[0]
            sections[cur] = []
        elif line.strip() and not line.startswith("#"):
            sections[cur].append([float(x) for x in line.split()])
    rec = np.array(sections["records"])
    got, chk = _ingest(psd, rec[:, 0].astype(np.int64), rec[:, 1:], (2, 1, 3), id_base=1)
    ref, once, rchk = orc.reorder_by_id(rec[:, 0].astype(np.int64), rec[:, 1:], (2, 1, 3),
                                        id_base=1)
    assert chk == rchk == (2, 1, 2)
    g, r = got.reshape(-1, 3), ref.reshape(-1, 3)
    assert np.array_equal(g[once], r[once])
    # the duplicated slot holds one of its two records; unnamed slots keep their fill
    assert any(np.array_equal(g[5], np.float32(x)) for x in ([0.125, 0.5, 0.375], [0.7, 0.7, 0.7]))
    assert np.isnan(g[[2, 4]]).all()


@pytest.mark.parametrize("np_, n_drop", [((32, 32, 32), 0), ((17, 9, 23), 5), ((64, 64, 64), 1)])
def test_ingest_permutation(psd, orc, np_, n_drop):
    """Seeded permutations of a Zel'dovich grid (ragged sizes, some records dropped so that
    slots go missing): bit-exact against the oracle, counts exact."""
    rng = np.random.default_rng(81)
    grid = zeldovich_positions(max(np_), 0.7, seed=82)[:np_[0], :np_[1], :np_[2]].copy()
    n = int(np.prod(np_))
    perm = rng.permutation(n)[: n - n_drop]
    rec = grid.reshape(-1, 3)[perm]
    got, chk = _ingest(psd, perm + 3, rec, np_, id_base=3)
    ref, once, rchk = orc.reorder_by_id(perm + 3, rec, np_, id_base=3)
    assert chk == rchk == (0, 0, n_drop)
    assert np.array_equal(got.reshape(-1, 3)[once], ref.reshape(-1, 3)[once])
    assert np.isnan(got.reshape(-1, 3)[~once]).all()


def test_ingest_bad_ids_and_duplicates(psd, orc):
    np_ = (20, 20, 20)
    rng = np.random.default_rng(83)
    n = 9000
    ids = rng.integers(-50, 8200, size=n)          # out of range, duplicates and gaps
    rec = rng.uniform(0, 1, size=(n, 3)).astype(np.float32)
    got, chk = _ingest(psd, ids, rec, np_)
    ref, once, rchk = orc.reorder_by_id(ids, rec, np_)
    assert chk == rchk
    assert rchk[0] > 0 and rchk[1] > 0 and rchk[2] > 0
    assert np.array_equal(got.reshape(-1, 3)[once], ref.reshape(-1, 3)[once])
    # every slot named more than once holds one of its records
    flat = got.reshape(-1, 3)
    for slot in np.nonzero(np.bincount(ids[(ids >= 0) & (ids < 8000)], minlength=8000) > 1)[0][:200]:
        cands = rec[ids == slot]
        assert any(np.array_equal(flat[slot], c) for c in cands)


def test_ingest_empty_and_unchecked(psd):
    got, chk = _ingest(psd, np.zeros(0, np.int64), np.zeros((0, 3), np.float32), (4, 4, 4))
    assert chk == (0, 0, 64) and np.isnan(got).all()
    # without the check the scatter alone runs
    dev = _dev()
    grid = zeldovich_positions(16, 0.5, seed=84)
    perm = np.random.default_rng(85).permutation(16 ** 3)
    out = psd.reorder_by_id(torch.from_numpy(perm).to(dev),
                            torch.from_numpy(grid.reshape(-1, 3)[perm]).to(dev), (16, 16, 16))
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), grid)


def test_ingest_full_size(psd):
    """The benchmark's 256^3 grid in a seeded random record order: the scatter restores it
    bit for bit (the definition at full size), and the check finds no fault."""
    pos, p = workload("zel256_g512")
    n = pos.shape[0] ** 3
    perm = np.random.default_rng(86).permutation(n)
    got, chk = _ingest(psd, perm, pos.reshape(-1, 3)[perm], pos.shape[:3])
    assert chk == (0, 0, 0)
    assert np.array_equal(got, pos)


# ---------------------------------------------------------------------------
# Coarse levels
# ---------------------------------------------------------------------------

def _rel_l1(a, b):
    return float(np.abs(a - b).sum() / max(np.abs(b).sum(), 1e-300))


def _rel_linf(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _block_sums(nodes, blocks, B, density):
    """Every internal node from its children's blocks (float64), bottom-up from `blocks`."""
    want = blocks.astype(np.float64).copy()
    h = B // 2
    for n in range(len(nodes)):
        fc = int(nodes["first_child"][n])
        if fc < 0:
            continue
        acc = np.zeros((B, B, B))
        for k in range(8):
            ch = nodes[fc + k]
            qx, qy, qz = int(ch["ix"]) & 1, int(ch["iy"]) & 1, int(ch["iz"]) & 1
            c = blocks[fc + k].astype(np.float64).reshape(h, 2, h, 2, h, 2).sum(axis=(1, 3, 5))
            acc[qx * h:(qx + 1) * h, qy * h:(qy + 1) * h, qz * h:(qz + 1) * h] = c
        want[n] = acc / 8.0 if density else acc
    return want


@pytest.mark.parametrize("density", [False, True])
def test_coarsen_against_oracle(psd, orc, density):
    pos = zeldovich_positions(16, 0.8, seed=87)
    dev = _dev()
    pt = torch.from_numpy(pos).to(dev)
    B = 4
    tree = psd.build_octree(pt, block=B, max_level=2, subblock=4, threshold=3000)
    nodes = tree.to_numpy()
    assert (nodes["first_child"] >= 0).sum() >= 2 and (nodes["level"] == 2).any()
    flags = psd.PSD_OUT_DENSITY if density else 0
    leaves = psd.deposit_octree(pt, tree, flags=flags)
    blocks = psd.octree_coarsen(tree, leaves, density=density)
    torch.cuda.synchronize()
    got = blocks.cpu().numpy()
    ref = orc.coarse_levels(pos, nodes, B, density=density)
    for n in range(len(nodes)):
        l1, linf = _rel_l1(got[n], ref[n]), _rel_linf(got[n], ref[n])
        assert l1 <= 1e-5 and linf <= 1e-5, (n, int(nodes["level"][n]), l1, linf)
    # internal nodes are the exact block sums of the GPU's own children
    want = _block_sums(nodes, got, B, density)
    internal = nodes["first_child"] >= 0
    assert np.allclose(got[internal], want[internal], rtol=4e-7, atol=0)
    # leaves copied bit for bit
    lv = leaves.cpu().numpy()
    for n in np.nonzero(~internal)[0]:
        assert np.array_equal(got[n], lv[int(nodes["leaf_id"][n])])
    if not density:
        assert abs(got[0].astype(np.float64).sum() - 1.0) <= 1e-5


def test_coarsen_single_leaf_and_errors(psd):
    pos = zeldovich_positions(8, 0.5, seed=88)
    dev = _dev()
    pt = torch.from_numpy(pos).to(dev)
    tree = psd.build_octree(pt, block=5, max_level=2, subblock=4, threshold=1 << 40)
    assert tree.n_nodes == 1
    leaves = psd.deposit_octree(pt, tree)
    blocks = psd.octree_coarsen(tree, leaves)
    torch.cuda.synchronize()
    assert np.array_equal(blocks.cpu().numpy()[0], leaves.cpu().numpy()[0])
    # an odd block cannot be halved: refused when the tree has internal nodes
    t2 = psd.build_octree(pt, block=5, max_level=1, subblock=4, threshold=10)
    assert t2.n_nodes > 1
    l2 = psd.deposit_octree(pt, t2)
    with pytest.raises(psd.PsdError) as e:
        psd.octree_coarsen(t2, l2)
    assert e.value.code == psd.PSD_ERR_UNSUPPORTED


@functools.lru_cache(maxsize=1)
def _clumps():
    return workload("clump512_octree")


def test_coarsen_full_size(psd):
    """512^3 particles + clumps: every internal node equals the block sums of its children,
    and the root holds the whole mass."""
    pos, p = _clumps()
    dev = _dev()
    pt = torch.from_numpy(pos).to(dev)
    tree = psd.build_octree(pt, block=p["block"], max_level=p["max_level"], subblock=8,
                            threshold=p["threshold"])
    leaves = psd.deposit_octree(pt, tree)
    blocks = psd.octree_coarsen(tree, leaves)
    torch.cuda.synchronize()
    nodes = tree.to_numpy()
    got = blocks.cpu().numpy()
    want = _block_sums(nodes, got, p["block"], False)
    internal = nodes["first_child"] >= 0
    assert np.allclose(got[internal], want[internal], rtol=4e-7, atol=1e-30)
    assert abs(got[0].astype(np.float64).sum() - 1.0) <= 1e-5
