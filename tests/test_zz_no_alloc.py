"""psd_deposit_uniform_noalloc (the deposit for callers that cannot allocate: its
workspace is the library's fixed per-GPU scratch array) against psd_deposit_uniform
with a caller workspace, through the C ABI, on two calls in a row, the second on a
smaller input.  Same kernels, other atomic order: an FP64 grid agrees to rounding,
an FP32 grid to the batched-versus-single bar; the integer counters agree exactly."""

import os

import numpy as np
import pytest
import torch

from synth import zeldovich_positions

pytestmark = pytest.mark.gpu

SURROGATE_WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                                 "paper_1612_09491_amd", "surrogate_zel256_g64.npy")


@pytest.fixture(scope="module")
def psd():
    import paper_1612_09491_amd as psd
    if not os.path.exists(psd.LIB_PATH):
        from paper_1612_09491_amd import build
        build.build()
    return psd


def _both(psd, pos, nc, flags, tuning=None, surrogate=None):
    dev = torch.device("cuda:0")
    pt = torch.from_numpy(np.ascontiguousarray(pos)).to(dev)
    res = []
    for fn in (psd.deposit_uniform, psd.deposit_uniform_noalloc):
        ms = torch.zeros(1, dtype=torch.float64, device=dev)
        st = torch.zeros(8, dtype=torch.int64, device=dev)
        out = fn(pt, nc, flags=flags, mass_sum=ms, stats=st, tuning=tuning, surrogate=surrogate)
        torch.cuda.synchronize()
        res.append((out.double().cpu().numpy(), float(ms.item()), st.cpu().numpy()))
    return res


def _rel_l1(a, b):
    return float(np.abs(a - b).sum() / np.abs(b).sum())


def _agree(ref, got, l1_bar, mass_bar):
    (g0, m0, s0), (g1, m1, s1) = ref, got
    l1 = _rel_l1(g1, g0)
    linf = float(np.abs(g1 - g0).max() / np.abs(g0).max())
    print(f"noalloc vs workspace: L1 {l1:.3e} Linf {linf:.3e} mass {abs(m1 - m0):.3e}", flush=True)
    assert l1 <= l1_bar and linf <= l1_bar
    assert abs(m1 - m0) <= mass_bar
    assert (s0 == s1).all(), (s0, s1)


def test_noalloc_matches_workspace_call_twice_in_a_row(psd):
    # first call: 32^3 -> 64^3, FP64 grid, chunks in cost order (buckets and order in scratch)
    big = zeldovich_positions(32, 0.5, seed=71)
    print("noalloc case 1: 32^3 -> 64^3 FP64 ordered", flush=True)
    r = _both(psd, big, 64, psd.PSD_PREC_FP64, tuning=(0, 0, 1))
    _agree(r[0], r[1], 1e-12, 1e-12)
    # second call, smaller: 12^3 -> 24^3, FP32 grid, positions checked first
    small = zeldovich_positions(12, 0.6, seed=72)
    print("noalloc case 2: 12^3 -> 24^3 FP32 checked", flush=True)
    r = _both(psd, small, 24, psd.PSD_CHECK_FINITE)
    _agree(r[0], r[1], 1e-6, 1e-12)


def test_noalloc_surrogate_mask_in_scratch(psd):
    # the surrogate's per-chunk mask of tets left to the exact pass sits in scratch
    w = torch.from_numpy(np.load(SURROGATE_WEIGHTS).astype(np.float32)).to("cuda:0")
    pos = zeldovich_positions(32, 2.0, seed=73)
    print("noalloc case 3: 32^3 -> 8^3 FP64 surrogate", flush=True)
    r = _both(psd, pos, 8, psd.PSD_PREC_FP64 | psd.PSD_SURROGATE, surrogate=w)
    assert r[0][2][6] > 0  # the network took some tets
    _agree(r[0], r[1], 1e-12, 1e-12)
    small = zeldovich_positions(16, 2.0, seed=74)
    print("noalloc case 4: 16^3 -> 4^3 FP64 surrogate", flush=True)
    r = _both(psd, small, 4, psd.PSD_PREC_FP64 | psd.PSD_SURROGATE, surrogate=w)
    _agree(r[0], r[1], 1e-12, 1e-12)


def test_noalloc_refuses_workspace_beyond_scratch(psd):
    # 256^3 particles in cost order need 12 bytes per 64 tets of order: more than 16 MiB.
    # The size check runs on the host before anything is enqueued.
    pt = torch.empty((256, 256, 256, 3), dtype=torch.float32, device="cuda:0")
    need = psd.uniform_workspace_size((256, 256, 256), 64, 0, tuning=(0, 0, 1))
    assert need > psd.PSD_NOALLOC_SCRATCH_BYTES
    out = torch.zeros((64, 64, 64), dtype=torch.float32, device="cuda:0")
    with pytest.raises(psd.PsdError) as e:
        psd.deposit_uniform_noalloc(pt, 64, out=out, tuning=(0, 0, 1))
    assert e.value.code == psd.PSD_ERR_WORKSPACE
    torch.cuda.synchronize()
    assert float(out.abs().sum().item()) == 0.0
