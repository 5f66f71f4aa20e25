"""GPU checks of the C ABI's input contract: non-finite positions (Section 2 takes
tracer positions in a periodic box; a NaN or infinity cannot be placed) and the
binding's refusal of side outputs that the kernels could not write safely.

With PSD_CHECK_FINITE every deposit (uniform, both methods; batched; octree)
returns PSD_ERR_NONFINITE and leaves its outputs untouched; psd_build_octree
always checks.  Without the flag, each tetrahedron with a bad vertex is dropped
and counted in stats[7]: one particle is a corner of 8 Lagrangian cubes and
belongs to 24 of their 48 tetrahedra (all 6 where it is corner 000 or 111, 2
where it is one of the other six corners).
"""

import numpy as np
import pytest
import torch

from synth import zeldovich_positions

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def psd():
    import os
    import paper_1612_09491_amd as psd
    if not os.path.exists(psd.LIB_PATH):
        from paper_1612_09491_amd import build
        build.build()
    return psd


def _bad_positions(n=8, value=np.nan, where=(3, 4, 5), axis=1):
    pos = zeldovich_positions(n, 0.6, seed=61)
    bad = pos.copy()
    bad[where + (axis,)] = value
    return pos, bad


@pytest.mark.parametrize("value", [np.nan, np.inf, -np.inf])
@pytest.mark.parametrize("method", [0, 8])  # default, PSD_METHOD_CELL
def test_uniform_check_finite_refuses(psd, value, method):
    _, bad = _bad_positions(value=value)
    dev = torch.device("cuda:0")
    pt = torch.from_numpy(bad).to(dev)
    out = torch.full((16, 16, 16), 7.0, dtype=torch.float32, device=dev)
    with pytest.raises(psd.PsdError) as e:
        psd.deposit_uniform(pt, 16, flags=psd.PSD_CHECK_FINITE | method, out=out)
    assert e.value.code == psd.PSD_ERR_NONFINITE
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())  # nothing was deposited


@pytest.mark.parametrize("method", [0, 8])
def test_uniform_drops_and_counts_without_the_flag(psd, orc, method):
    good, bad = _bad_positions()
    dev = torch.device("cuda:0")
    ms = torch.zeros(1, dtype=torch.float64, device=dev)
    st = torch.zeros(8, dtype=torch.int64, device=dev)
    out = psd.deposit_uniform(torch.from_numpy(bad).to(dev), 16, flags=method, mass_sum=ms, stats=st)
    torch.cuda.synchronize()
    s = st.cpu().numpy()
    m = 1.0 / (6 * 8 ** 3)
    assert s[7] == 24 and s[0] == 6 * 8 ** 3
    # the per-cell method sums its FP32 cell values in FP64; the default sums FP64 pieces
    tol = 1e-12 if method == 0 else 1e-6
    assert abs(float(ms.item()) - (1.0 - 24 * m)) <= tol
    got = out.double().cpu().numpy()
    assert np.isfinite(got).all()
    assert abs(got.sum() - (1.0 - 24 * m)) <= 1e-5
    # the same call with finite positions drops nothing
    st.zero_()
    psd.deposit_uniform(torch.from_numpy(good).to(dev), 16, flags=method | psd.PSD_CHECK_FINITE,
                        stats=st)
    torch.cuda.synchronize()
    assert int(st[7].item()) == 0


def test_batched_check_finite(psd):
    good, bad = _bad_positions()
    dev = torch.device("cuda:0")
    g = torch.from_numpy(good).to(dev)
    b = torch.from_numpy(bad).to(dev)
    with pytest.raises(psd.PsdError) as e:
        psd.deposit_batched([(g, 16), (b, 12)], flags=psd.PSD_CHECK_FINITE)
    assert e.value.code == psd.PSD_ERR_NONFINITE
    st = torch.zeros(8, dtype=torch.int64, device=dev)
    ms = torch.zeros(2, dtype=torch.float64, device=dev)
    psd.deposit_batched([(g, 16), (b, 12)], mass_sums=ms, stats=st)
    torch.cuda.synchronize()
    m = 1.0 / (6 * 8 ** 3)
    assert int(st[7].item()) == 24
    assert abs(float(ms[0].item()) - 1.0) <= 1e-12
    assert abs(float(ms[1].item()) - (1.0 - 24 * m)) <= 1e-12


def test_octree_checks(psd):
    good, bad = _bad_positions(n=16)
    dev = torch.device("cuda:0")
    g = torch.from_numpy(good).to(dev)
    b = torch.from_numpy(bad).to(dev)
    kw = dict(block=4, max_level=2, subblock=4, threshold=2000)
    with pytest.raises(psd.PsdError) as e:
        psd.build_octree(b, **kw)
    assert e.value.code == psd.PSD_ERR_NONFINITE
    tree = psd.build_octree(g, **kw)
    with pytest.raises(psd.PsdError) as e:
        psd.deposit_octree(b, tree, flags=psd.PSD_CHECK_FINITE)
    assert e.value.code == psd.PSD_ERR_NONFINITE
    st = torch.zeros(8, dtype=torch.int64, device=dev)
    ms = torch.zeros(1, dtype=torch.float64, device=dev)
    psd.deposit_octree(b, tree, stats=st, mass_sum=ms)
    torch.cuda.synchronize()
    levels = np.unique(tree.to_numpy()["level"][tree.to_numpy()["leaf_id"] >= 0]).size
    # one walk per level that has leaves
    assert int(st[7].item()) == 24 * levels
    m = 1.0 / (6 * 16 ** 3)
    assert abs(float(ms.item()) - (1.0 - 24 * m)) <= 1e-12


def test_binding_refuses_bad_side_outputs(psd):
    pos = zeldovich_positions(8, 0.6, seed=62)
    dev = torch.device("cuda:0")
    pt = torch.from_numpy(pos).to(dev)
    tree = psd.build_octree(pt, block=4, max_level=1, subblock=4, threshold=10)
    bad_sums = [torch.zeros(1, dtype=torch.float32, device=dev), torch.zeros(1, dtype=torch.float64)]
    bad_stats = [torch.zeros(8, dtype=torch.int32, device=dev),
                 torch.zeros(4, dtype=torch.int64, device=dev)]
    for ms in bad_sums:
        with pytest.raises(ValueError):
            psd.deposit_octree(pt, tree, mass_sum=ms)
        with pytest.raises(ValueError):
            psd.deposit_batched([(pt, 16)], mass_sums=ms)
    for st in bad_stats:
        with pytest.raises(ValueError):
            psd.deposit_octree(pt, tree, stats=st)
        with pytest.raises(ValueError):
            psd.deposit_batched([(pt, 16)], stats=st)
    with pytest.raises(ValueError):
        psd.deposit_batched([(pt, 16), (pt, 8)], mass_sums=torch.zeros(1, dtype=torch.float64,
                                                                         device=dev))
    with pytest.raises(ValueError):
        psd.deposit_octree(pt, tree, out=torch.zeros((tree.n_leaves, 4, 4, 4)))  # host memory
    with pytest.raises(ValueError):
        psd.deposit_uniform(pt, 16, workspace=torch.zeros(8, dtype=torch.uint8, device=dev))
