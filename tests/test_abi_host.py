"""Host-side checks of the C ABI (no GPU work is launched).

The library must load, export every function declared in include/psd.h, and
reject bad arguments on the host before touching the device.
"""

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def psd():
    import paper_1612_09491_amd as psd
    if not os.path.exists(psd.LIB_PATH):
        from paper_1612_09491_amd import build
        build.build()
    return psd


def _declared_functions():
    names = []
    for hdr in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not hdr.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", hdr)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"\b(psd_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_every_declared_symbol_is_exported(psd):
    names = _declared_functions()
    assert "psd_deposit_uniform" in names and len(names) >= 4
    L = C.CDLL(psd.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_status_strings(psd):
    L = psd.lib()
    assert L.psd_status_string(0) == b"PSD_OK"
    assert L.psd_status_string(-2) == b"PSD_ERR_WORKSPACE"


def test_workspace_size_and_argument_errors(psd):
    assert psd.uniform_workspace_size((8, 8, 8), 16) > 0
    with pytest.raises(psd.PsdError) as e:
        psd.uniform_workspace_size((0, 8, 8), 16)
    assert e.value.code == psd.PSD_ERR_ARG
    with pytest.raises(psd.PsdError) as e:
        psd.uniform_workspace_size((8, 8, 8), (16, 0, 16))
    assert e.value.code == psd.PSD_ERR_ARG
    with pytest.raises(psd.PsdError) as e:
        psd.uniform_workspace_size((8, 8, 8), 16, flags=1 << 20)
    assert e.value.code == psd.PSD_ERR_UNSUPPORTED
    # the per-cell method numbers bbox cells in 32 bits: refused where a bbox could overflow
    assert psd.uniform_workspace_size((8, 8, 8), 1289, flags=psd.PSD_METHOD_CELL) > 0
    with pytest.raises(psd.PsdError) as e:
        psd.uniform_workspace_size((8, 8, 8), 1290, flags=psd.PSD_METHOD_CELL)
    assert e.value.code == psd.PSD_ERR_UNSUPPORTED
    assert psd.uniform_workspace_size((8, 8, 8), 1290) > 0  # the default method has no limit
    # the surrogate flag needs the default method and parameters
    with pytest.raises(psd.PsdError):
        L = psd.lib()
        p = psd.Particles()
        for a in range(3):
            p.np[a] = 4
        p.box, p.total_mass = 1.0, 1.0
        nc = (C.c_int32 * 3)(8, 8, 8)
        o = psd.Options(psd.PSD_SURROGATE, None, None, None)
        fake = C.c_void_p(0x1000)
        psd._check(L.psd_deposit_uniform(fake, C.byref(p), nc, fake, None, C.byref(o), fake,
                                          1 << 30, None), "psd_deposit_uniform")


def test_deposit_rejects_bad_arguments_before_launch(psd):
    L = psd.lib()
    p = psd.Particles()
    for a in range(3):
        p.np[a] = 4
    p.box, p.total_mass = 1.0, 1.0
    nc = (C.c_int32 * 3)(8, 8, 8)
    o = psd.Options(0, None)
    fake = C.c_void_p(0x1000)  # never dereferenced: checks fail first
    assert L.psd_deposit_uniform(None, C.byref(p), nc, fake, None, C.byref(o), fake, 4096,
                                 None) == psd.PSD_ERR_ARG
    assert L.psd_deposit_uniform(fake, C.byref(p), nc, fake, None, C.byref(o), fake, 1,
                                 None) == psd.PSD_ERR_WORKSPACE
    assert L.psd_deposit_uniform(fake, C.byref(p), nc, fake, None, C.byref(o), None, 4096,
                                 None) == psd.PSD_ERR_WORKSPACE
    p.box = -1.0
    assert L.psd_deposit_uniform(fake, C.byref(p), nc, fake, None, C.byref(o), fake, 4096,
                                 None) == psd.PSD_ERR_ARG
    assert b"particle" in L.psd_last_error_detail()


def test_launch_shape_validation(psd):
    # buffer sizes are the kernel's instances; 0 means the defaults (chosen from
    # the grid's cells per spacing, as many wavefronts as fit a compute unit)
    for cap in (0, 512, 960, 1024, 1408, 2048):
        assert psd.uniform_workspace_size((8, 8, 8), 16, tuning=(cap, 0, 0)) > 0
    for bad in ((1000, 0, 0), (960, -1, 0), (960, 65, 0)):
        with pytest.raises(psd.PsdError) as e:
            psd.uniform_workspace_size((8, 8, 8), 16, tuning=bad)
        assert e.value.code == psd.PSD_ERR_ARG


def test_float_reciprocal_quotient_is_exact():
    """The deposit kernel divides indices n < 2^21 (columns of a tile, cells
    of a group tile, grid cells plus a tile offset) by integers d up to 2^20
    (a tile's width, a leaf side, a grid side) as trunc((n + 1/2) * r) in
    FP32, r the hardware reciprocal of d (within one ulp of 1/d): the error
    stays below the 1/(2d) that separates (n + 1/2)/d from an integer, so the
    quotient is exact.  Checked here with IEEE FP32 arithmetic for every n and
    for 1/d rounded to float and one ulp either side."""
    import numpy as np
    n = np.arange(1 << 21, dtype=np.int64)
    nf = n.astype(np.float32) + np.float32(0.5)
    rng = np.random.default_rng(7)
    ds = sorted(set(range(1, 65)) | {1 << k for k in range(21)} | {4095, 4093, 3001, 2047}
                | set(int(d) for d in rng.integers(65, 4097, 60))
                | set(int(d) for d in rng.integers(4097, (1 << 20) + 1, 20)))
    for d in ds:
        r = np.float32(1.0 / d)
        for inv in (r, np.nextafter(r, np.float32(0)), np.nextafter(r, np.float32(1))):
            q = (nf * inv).astype(np.int64)
            assert np.array_equal(q, n // d), (d, inv)


def test_octree_leaf_side_limit(psd):
    # cells within a leaf are indexed in 32 bits: leaves of up to 1024^3 cells
    assert psd.octree_workspace_size((8, 8, 8), block=1024, max_level=0) > 0
    with pytest.raises(psd.PsdError) as e:
        psd.octree_workspace_size((8, 8, 8), block=1025, max_level=0)
    assert e.value.code == psd.PSD_ERR_ARG


def test_wrapper_rejects_bad_side_outputs(psd):
    """Mass sums and counters receive 8-byte device atomics: anything that is not a CUDA
    float64 (int64) tensor of the right length is refused before a call is made."""
    import torch
    with pytest.raises(ValueError):
        psd._check_aux(torch.zeros(1, dtype=torch.float32), 1, None)
    with pytest.raises(ValueError):
        psd._check_aux(torch.zeros(1, dtype=torch.float64), 1, None)  # host memory
    with pytest.raises(ValueError):
        psd._check_aux(None, 1, torch.zeros(8, dtype=torch.int32))
    with pytest.raises(ValueError):
        psd._check_aux(None, 1, torch.zeros(4, dtype=torch.int64))
    with pytest.raises(ValueError):
        psd._check_aux(None, 1, torch.zeros(8, dtype=torch.int64))  # host memory
    with pytest.raises(ValueError):
        psd._workspace(torch.zeros(16, dtype=torch.uint8), 8, None)  # host memory
    psd._check_aux(None, 3, None)


def test_check_finite_flag_is_accepted(psd):
    """PSD_CHECK_FINITE is a known flag of every deposit; unknown bits are refused."""
    assert psd.PSD_CHECK_FINITE == 1 << 5
    assert psd.uniform_workspace_size((8, 8, 8), 16, flags=psd.PSD_CHECK_FINITE) > 0
    assert psd.STAT_NAMES[7] == "dropped_nonfinite"


def test_slab_flag_combinations(psd):
    """PSD_METHOD_SLAB (FP32 cell volumes) is accepted alone and with the output flags, and
    refused with an FP64 grid, the per-cell method, the surrogate or the work counters."""
    assert psd.PSD_METHOD_SLAB == 1 << 7
    ok = (0, psd.PSD_OUT_DENSITY, psd.PSD_ACCUMULATE, psd.PSD_CHECK_FINITE)
    for extra in ok:
        assert psd.uniform_workspace_size((8, 8, 8), 16, flags=psd.PSD_METHOD_SLAB | extra) > 0
    for bad in (psd.PSD_PREC_FP64, psd.PSD_METHOD_CELL, psd.PSD_SURROGATE, psd.PSD_WORK_COUNTERS):
        with pytest.raises(psd.PsdError) as e:
            psd.uniform_workspace_size((8, 8, 8), 16, flags=psd.PSD_METHOD_SLAB | bad)
        assert e.value.code == psd.PSD_ERR_UNSUPPORTED


def test_train_steps_rejects_bad_arguments_before_launch(psd):
    L = psd.lib()
    psd._bind_surrogate(L)
    f = C.c_void_p(0x1000)  # never dereferenced: checks fail first

    def call(n=1000, batch=256, steps=4, step0=0, b1=0.9, b2=0.999, eps=1e-8, ptr=f):
        return L.psd_surrogate_train_steps(ptr, f, f, f, f, n, batch, steps, step0, f, b1, b2,
                                           eps, f, f, f, None, None)

    assert call(steps=0) == psd.PSD_OK  # nothing to do, nothing launched
    assert call(batch=0) == psd.PSD_ERR_ARG
    assert call(steps=-1) == psd.PSD_ERR_ARG
    assert call(step0=-1) == psd.PSD_ERR_ARG
    assert call(steps=5) == psd.PSD_ERR_ARG  # 1000 samples hold 4 batches of 256
    assert b"more steps" in L.psd_last_error_detail()
    assert call(b1=1.0) == psd.PSD_ERR_ARG
    assert call(eps=0.0) == psd.PSD_ERR_ARG
    assert call(ptr=None) == psd.PSD_ERR_ARG
