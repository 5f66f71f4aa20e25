"""GPU parity of psd_deposit_uniform against the FP64 oracle.

Three methods are checked: the default cumulative method (FP64 arithmetic),
the per-cell cell-local FP32 clip (PSD_METHOD_CELL) and the cached slab clip in
FP32 (PSD_METHOD_SLAB).  Tolerances: an FP32 output grid or FP32 clipping
within 1e-5 relative L1 and Linf of the oracle's densities; FP64 arithmetic
into an FP64 grid within 1e-12.  Integer counters (tets, bbox pairs, inverted,
zero-volume) must match exactly.
"""

import functools

import numpy as np
import pytest
import torch

from synth import lattice_positions, zeldovich_positions, workload

pytestmark = pytest.mark.gpu

FP32_L1 = 1e-5
FP32_LINF = 1e-5
FP64_L1 = 1e-12
FP64_LINF = 1e-11


@pytest.fixture(scope="module")
def psd():
    import os
    import paper_1612_09491_amd as psd
    if not os.path.exists(psd.LIB_PATH):
        from paper_1612_09491_amd import build
        build.build()
    return psd


def _run(psd, pos, nc, flags=0, box=1.0, mass=1.0):
    dev = torch.device("cuda:0")
    pt = torch.from_numpy(np.ascontiguousarray(pos)).to(dev)
    ms = torch.zeros(1, dtype=torch.float64, device=dev)
    st = torch.zeros(8, dtype=torch.int64, device=dev)
    out = psd.deposit_uniform(pt, nc, box=box, mass=mass, flags=flags, mass_sum=ms, stats=st)
    torch.cuda.synchronize()
    return out.double().cpu().numpy(), float(ms.item()), st.cpu().numpy()


def _rel_l1(a, b):
    return float(np.abs(a - b).sum() / np.abs(b).sum())


def _rel_linf(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _check_stats(st, cnt):
    assert st[0] == cnt["n_tet"]
    assert st[1] == cnt["n_pair"]
    assert st[4] == cnt["n_inverted"]
    assert st[5] == cnt["n_degenerate"]


METHODS = {"cumulative": 0, "cell": 8, "slab": 128}  # PSD_METHOD_CELL, PSD_METHOD_SLAB
FP64_METHODS = {"cumulative": 0, "cell": 8}  # the methods with FP64 arithmetic into FP64 grids


@pytest.mark.parametrize("method", list(METHODS))
@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_zel32_g64_fp32(psd, orc, seed, method):
    pos, p = workload("zel32_g64", seed=seed)
    ref, cnt = orc.deposit_uniform(pos, p["nc"])
    got, msum, st = _run(psd, pos, p["nc"], flags=METHODS[method])
    l1, linf = _rel_l1(got, ref), _rel_linf(got, ref)
    print(f"seed {seed}: L1 {l1:.3e} Linf {linf:.3e} mass {msum - 1:.3e}")
    assert l1 <= FP32_L1 and linf <= FP32_LINF
    assert abs(msum - 1.0) <= 1e-6
    _check_stats(st, cnt)


@pytest.mark.parametrize("method", list(FP64_METHODS))
@pytest.mark.parametrize("seed", [1, 2])
def test_zel32_g64_fp64(psd, orc, seed, method):
    pos, p = workload("zel32_g64", seed=seed)
    ref, cnt = orc.deposit_uniform(pos, p["nc"])
    got, msum, st = _run(psd, pos, p["nc"], flags=psd.PSD_PREC_FP64 | FP64_METHODS[method])
    assert _rel_l1(got, ref) <= FP64_L1 and _rel_linf(got, ref) <= FP64_LINF
    assert abs(msum - 1.0) <= 1e-12
    _check_stats(st, cnt)


@pytest.mark.parametrize("method", list(METHODS))
@pytest.mark.parametrize("nc", [64, 16, 24])
def test_undisplaced_lattice_is_uniform(psd, nc, method):
    pos = lattice_positions(32)
    got, _, st = _run(psd, pos, nc, flags=METHODS[method])
    assert np.max(np.abs(got * nc ** 3 - 1.0)) <= 1e-5
    if method in FP64_METHODS:
        got64, _, _ = _run(psd, pos, nc, flags=psd.PSD_PREC_FP64 | METHODS[method])
        assert np.max(np.abs(got64 * nc ** 3 - 1.0)) <= 1e-12


def _compare(psd, orc, pos, nc, box=1.0, mass=1.0, l1=FP32_L1):
    ref, cnt = orc.deposit_uniform(pos, nc, box=box, mass=mass)
    for m in METHODS.values():
        got, msum, st = _run(psd, pos, nc, box=box, mass=mass, flags=m)
        assert _rel_l1(got, ref) <= l1, (m, _rel_l1(got, ref))
        _check_stats(st, cnt)
        if m not in FP64_METHODS.values():
            continue
        got64, msum64, _ = _run(psd, pos, nc, flags=psd.PSD_PREC_FP64 | m, box=box, mass=mass)
        assert _rel_l1(got64, ref) <= FP64_L1, (m, _rel_l1(got64, ref))
        assert abs(msum64 - mass) <= 1e-12 * abs(mass)
    return got, ref


def test_single_particle_grid(psd, orc):
    pos = np.array([[[[0.3, 0.6, 0.9]]]], dtype=np.float32)
    got, ref = _compare(psd, orc, pos, 8)
    assert got[2, 4, 7] == pytest.approx(1.0)


def test_single_cell_grid(psd, orc):
    pos = zeldovich_positions(6, 0.7, seed=41)
    got, ref = _compare(psd, orc, pos, 1)
    # 1296 tets land in the one FP32 cell through atomics: n*u bounds the
    # rounding at ~8e-5, the FP32 tolerance of the other tests is tighter.
    assert got[0, 0, 0] == pytest.approx(1.0, rel=FP32_LINF)


def test_anisotropic_ragged_grids(psd, orc):
    rng = np.random.default_rng(42)
    q = np.moveaxis(np.indices((3, 5, 2), dtype=np.float64), 0, -1) / np.array([3, 5, 2])
    pos = np.mod(q + rng.normal(scale=0.05, size=q.shape), 1.0).astype(np.float32)
    _compare(psd, orc, pos, (7, 9, 4))
    pos2 = zeldovich_positions(10, 0.8, seed=43)
    _compare(psd, orc, pos2, (37, 20, 13))


def test_huge_stretched_tets(psd, orc):
    pos = zeldovich_positions(4, 1.4, seed=44)
    _compare(psd, orc, pos, 48)


def _max_bbox_cells(orc, pos, nc):
    """Largest bounding-box cell count over the tetrahedra (oracle's unwrapped vertices)."""
    n = pos.shape[0]
    best = 0
    for i in range(n):
        for j in range(n):
            for k in range(n):
                v, _ = orc.cube_tets(pos, (nc, nc, nc), i, j, k)
                e = np.floor(v.max(axis=1)) - np.floor(v.min(axis=1)) + 1
                best = max(best, int(np.prod(e, axis=1).max()))
    return best


@pytest.mark.parametrize("tuning", [(512, 0, 0), (960, 0, 1), (1024, 0, 0), (1408, 0, 0),
                                    (2048, 0, 0)])
def test_huge_tets_tiled_in_every_instance(psd, orc, tuning):
    # tets of thousands of bbox cells are tiled with halo columns; in the 16-tet
    # instances they also interrupt the all-lanes planning of untiled runs
    pos = zeldovich_positions(4, 1.4, seed=44)
    # the input has tetrahedra whose bbox (the D array of the walk) exceeds the
    # instance's LDS buffer, so the tiled walk runs
    biggest = _max_bbox_cells(orc, pos, 48)
    assert biggest > tuning[0], (biggest, tuning)
    ref, _ = orc.deposit_uniform(pos, 48)
    dev = torch.device("cuda:0")
    pt = torch.from_numpy(pos).to(dev)
    st = torch.zeros(8, dtype=torch.int64, device=dev)
    out = psd.deposit_uniform(pt, 48, flags=psd.PSD_PREC_FP64, stats=st, tuning=tuning)
    assert _rel_l1(out.cpu().numpy(), ref) <= FP64_L1
    assert int(st[0].item()) == 6 * 4 ** 3


def test_huge_tets_tiled_in_the_slab_form(psd, orc):
    """The slab form tiles tetrahedra whose bbox exceeds its 2048-entry buffer or its 16
    cached rows: the FP32 cell volumes still meet the FP32 bar, whose error does not grow
    with the tetrahedron's size (no differences of cumulative values)."""
    pos = zeldovich_positions(4, 1.4, seed=44)
    biggest = _max_bbox_cells(orc, pos, 48)
    assert biggest > 2048, biggest
    ref, _ = orc.deposit_uniform(pos, 48)
    got, msum, st = _run(psd, pos, 48, flags=psd.PSD_METHOD_SLAB)
    l1, linf = _rel_l1(got, ref), _rel_linf(got, ref)
    print(f"slab, tets up to {biggest} bbox cells: L1 {l1:.3e} Linf {linf:.3e} mass {msum - 1:.3e}")
    assert l1 <= FP32_L1 and linf <= FP32_LINF
    assert abs(msum - 1.0) <= 1e-6


def test_zel64_g16_full_grid(psd, orc):
    """64^3 particles (rms 2 spacings) onto 16^3 cells, 0.25 cells per spacing: the
    geometry of the surrogate's workload at a size the oracle finishes in seconds;
    whole grid, FP32 and FP64 outputs."""
    pos, p = workload("zel64_g16")
    ref, cnt = orc.deposit_uniform(pos, p["nc"])
    got, msum, st = _run(psd, pos, p["nc"])
    l1, linf = _rel_l1(got, ref), _rel_linf(got, ref)
    print(f"zel64_g16 FP32 grid: L1 {l1:.3e} Linf {linf:.3e}")
    assert l1 <= FP32_L1 and linf <= FP32_LINF
    assert abs(msum - 1.0) <= 1e-12
    _check_stats(st, cnt)
    got64, msum64, _ = _run(psd, pos, p["nc"], flags=psd.PSD_PREC_FP64)
    l1, linf = _rel_l1(got64, ref), _rel_linf(got64, ref)
    print(f"zel64_g16 FP64 grid: L1 {l1:.3e} Linf {linf:.3e}")
    assert l1 <= FP64_L1 and linf <= FP64_LINF


def test_flat_tets_go_to_centroid_cell(psd, orc):
    pos = lattice_positions(8).astype(np.float64)
    pos[:, :, :, 2] = 0.3
    got, ref = _compare(psd, orc, pos.astype(np.float32), 8)
    assert np.count_nonzero(got.sum(axis=(0, 1))) == 1


def test_images_outside_the_box(psd, orc):
    pos = zeldovich_positions(10, 0.9, seed=45)
    q = (np.round(pos.astype(np.float64) * 2 ** 16) / 2 ** 16).astype(np.float32)
    rng = np.random.default_rng(46)
    shift = rng.integers(-3, 4, size=q.shape[:3] + (1,)).astype(np.float32)
    moved = (q + shift).astype(np.float32)
    assert np.array_equal(np.mod(moved.astype(np.float64), 1.0).astype(np.float32), q)
    a, _, _ = _run(psd, q, 20)
    b, _, _ = _run(psd, moved, 20)
    assert _rel_l1(b, a) <= 1e-6


def test_box_and_mass_scaling(psd, orc):
    pos = (zeldovich_positions(8, 0.7, seed=47).astype(np.float64) * 2.5).astype(np.float32)
    _compare(psd, orc, pos, 16, box=2.5, mass=7.0)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_density_and_accumulate_flags(psd, prec):
    """PSD_OUT_DENSITY divides by the cell volume; PSD_ACCUMULATE adds onto the
    caller's grid.  Separate runs add their FP32 atomics in different orders,
    so the FP32 grid is held to the FP32 tolerance and the FP64 grid to 1e-12."""
    pos = zeldovich_positions(8, 0.7, seed=48)
    nc = 16
    fp64 = prec == "fp64"
    pflag = psd.PSD_PREC_FP64 if fp64 else 0
    tol = 1e-12 if fp64 else FP32_LINF
    mass, _, _ = _run(psd, pos, nc, box=2.0, flags=pflag)
    dens, _, _ = _run(psd, pos, nc, box=2.0, flags=psd.PSD_OUT_DENSITY | pflag)
    h3 = (2.0 / nc) ** 3
    scale = mass.max()
    assert np.allclose(dens * h3, mass, rtol=tol, atol=tol * scale)
    dev = torch.device("cuda:0")
    pt = torch.from_numpy(pos).to(dev)
    base = 1e-3
    out = torch.full((nc, nc, nc), base, dtype=torch.float64 if fp64 else torch.float32, device=dev)
    psd.deposit_uniform(pt, nc, box=2.0, flags=psd.PSD_ACCUMULATE | pflag, out=out)
    psd.deposit_uniform(pt, nc, box=2.0, flags=psd.PSD_ACCUMULATE | pflag, out=out)
    torch.cuda.synchronize()
    base_eff = base if fp64 else float(np.float32(base))
    assert np.allclose(out.double().cpu().numpy(), base_eff + 2 * mass, rtol=tol, atol=tol * scale)


@functools.lru_cache(maxsize=1)
def _zel256():
    return workload("zel256_g512")


@pytest.mark.parametrize("method", list(METHODS))
def test_zel256_g512_sampled_blocks(psd, orc, method):
    """Full size (100.7M tets -> 512^3): oracle on sampled 16^3 blocks, global mass."""
    pos, p = _zel256()
    nc = p["nc"]
    got, msum, st = _run(psd, pos, nc, flags=METHODS[method])
    assert st[0] == 6 * 256 ** 3
    assert abs(msum - 1.0) <= 1e-6
    assert abs(got.sum() - 1.0) <= 1e-5
    rng = np.random.default_rng(2)
    for _ in range(8):
        lo = [int(x) for x in rng.integers(0, nc - 16, size=3)]
        ref, _ = orc.deposit_uniform(pos, nc, region=(lo, (16, 16, 16)))
        blk = got[lo[0]:lo[0] + 16, lo[1]:lo[1] + 16, lo[2]:lo[2] + 16]
        l1, linf = _rel_l1(blk, ref), _rel_linf(blk, ref)
        print(f"block {lo}: L1 {l1:.3e} Linf {linf:.3e}", flush=True)
        assert l1 <= FP32_L1 and linf <= FP32_LINF


@pytest.mark.parametrize("nc", [64, 20])
def test_kernel_instances_agree(psd, orc, nc):
    # 32^3 particles onto 64^3 (2 cells per spacing: the default is the 1024-entry
    # buffer with 8-tet groups) and onto 20^3 (0.6: 960 entries, 16-tet groups);
    # every instance and launch shape gives the oracle's grid in FP64
    pos = zeldovich_positions(32, 0.5, seed=9)
    ref, _ = orc.deposit_uniform(pos, nc)
    dev = torch.device("cuda:0")
    pt = torch.from_numpy(pos).to(dev)
    for tuning in (None, (512, 0, 0), (960, 12, 1), (1024, 12, 0), (1024, 4, 1), (1408, 12, 0),
                   (2048, 7, 0), (1408, 3, 1)):
        ms = torch.zeros(1, dtype=torch.float64, device=dev)
        out = psd.deposit_uniform(pt, nc, flags=psd.PSD_PREC_FP64, mass_sum=ms, tuning=tuning)
        got = out.cpu().numpy()
        assert _rel_l1(got, ref) <= FP64_L1, (tuning, _rel_l1(got, ref))
        assert abs(float(ms.item()) - 1.0) <= 1e-12


@pytest.mark.parametrize("cap", [1024, 1408, 960])
def test_work_counters_match_cost_model(psd, orc, cap):
    """The instrumented kernel's work events (PSD_WORK_COUNTERS) equal the CPU replay of
    the cumulative walk in costmodel.py on every tetrahedron of 32^3 -> 64^3; the split
    and level counts may differ only where rounding decides an on-plane vertex.  Its grid
    is held to the same parity bar as the plain kernel's."""
    import costmodel
    pos, p = workload("zel32_g64", seed=1)
    dev = torch.device("cuda:0")
    pt = torch.from_numpy(pos).to(dev)
    st = torch.zeros(16, dtype=torch.int64, device=dev)
    out = psd.deposit_uniform(pt, p["nc"], flags=psd.PSD_WORK_COUNTERS, stats=st,
                              tuning=(cap, 0, 0))
    torch.cuda.synchronize()
    s = st.cpu().numpy()
    cm = costmodel.count_events(pos, p["nc"], np.arange(32 ** 3), cap=cap)
    gpu = {"column": s[2], "xpiece": s[8], "piece": s[9], "level": s[10], "colcell": s[11]}
    print({k: (int(v), cm[k]) for k, v in gpu.items()})
    assert gpu["column"] == cm["column"] and gpu["colcell"] == cm["colcell"]
    for k in ("xpiece", "piece", "level"):
        assert abs(int(gpu[k]) - cm[k]) <= 1e-5 * cm[k] + 2, k
    ref, _ = orc.deposit_uniform(pos, p["nc"])
    got = out.double().cpu().numpy()
    assert _rel_l1(got, ref) <= FP32_L1 and _rel_linf(got, ref) <= FP32_LINF


@pytest.mark.parametrize("cap", [1024, 1408])
def test_work_counters_match_cost_model_tiled(psd, orc, cap):
    """The same on tetrahedra of thousands of bbox cells (4^3 particles -> 48^3 cells),
    which are tiled with halo rows and columns: the replay's tile shapes, halos, vertex
    order, frame choice and complement walks (x only in tiles that hold the bbox's last
    row) give the kernel's counts, and the FP64 grid meets the FP64 bar."""
    import costmodel
    pos = zeldovich_positions(4, 1.4, seed=44)
    dev = torch.device("cuda:0")
    pt = torch.from_numpy(pos).to(dev)
    st = torch.zeros(16, dtype=torch.int64, device=dev)
    out = psd.deposit_uniform(pt, 48, flags=psd.PSD_WORK_COUNTERS | psd.PSD_PREC_FP64, stats=st,
                              tuning=(cap, 0, 0))
    torch.cuda.synchronize()
    s = st.cpu().numpy()
    cm = costmodel.count_events(pos, 48, np.arange(4 ** 3), cap=cap)
    gpu = {"column": s[2], "xpiece": s[8], "piece": s[9], "level": s[10], "colcell": s[11]}
    print({k: (int(v), cm[k]) for k, v in gpu.items()})
    assert cm["colcell"] > 4 * cap  # tiles of several tets' worth of cells
    assert gpu["column"] == cm["column"] and gpu["colcell"] == cm["colcell"]
    for k in ("xpiece", "piece", "level"):
        assert abs(int(gpu[k]) - cm[k]) <= 1e-5 * cm[k] + 2, k
    ref, _ = orc.deposit_uniform(pos, 48)
    assert _rel_l1(out.cpu().numpy(), ref) <= FP64_L1
