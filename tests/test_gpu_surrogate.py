"""GPU parity of the learned overlap surrogate against the FP64 oracle.

- examples: eligibility, features and cell masks bit-identical to the oracle's,
  exact fractions within 1e-10 (both FP64, different clippers);
- forward / backward: the network on the GPU (BF16 matrix cores, FP32
  accumulate, BF16 activations between layers) against the FP64 reference on
  the same BF16-rounded weights: relative norm <= 1e-2, for the whole output
  and for every parameter block (measured: forward 4e-5, or 2e-3 with
  weights three times larger; gradient 6e-5, blocks below 3e-4);
- Adam: FP32 update against the FP64 reference, relative 1e-5;
- deposit: the surrogate deposit equals the oracle's composition (exact for
  the other tetrahedra, the FP64 reference network for the eligible ones),
  conserves mass, and counts the eligible tetrahedra;
- exact fractions of caller-given tetrahedra in a 2x2x2 block: the oracle's
  polytope clipper within 1e-10, rows summing to 1, the zero-volume rule and
  NaN rows for vertices outside the block.
"""

import math

import numpy as np
import pytest
import torch

from oracle import surrogate as S
from synth import TRAIN_SEED0, uniform_segments, workload, zeldovich_positions

pytestmark = pytest.mark.gpu

NET_TOL = 1e-2


@pytest.fixture(scope="module")
def psd():
    import os
    import paper_1612_09491_amd as psd
    if not os.path.exists(psd.LIB_PATH):
        from paper_1612_09491_amd import build
        build.build()
    return psd


def _theta(seed=3, scale=1.0):
    fan = {"W1": 12, "b1": 12, "W2": 64, "b2": 64, "W3": 64, "b3": 64, "W4": 64, "b4": 64}
    return uniform_segments([(int(np.prod(sh)), scale / math.sqrt(fan[n])) for n, sh in S.LAYOUT],
                            seed)


def _dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


@pytest.mark.parametrize("min_cells", [1, 2])
def test_examples_match_oracle(psd, orc, min_cells):
    pos = zeldovich_positions(16, 2.0, seed=61)
    nc = 4
    ref = orc.surrogate_examples(pos, nc)
    keep = np.array([bin(int(m)).count("1") >= min_cells for m in ref["mask"]], dtype=bool)
    ref = {k: v[keep] for k, v in ref.items()}
    got = psd.surrogate_examples(_dev(pos), nc, min_cells=min_cells)
    assert got["found"] == len(ref["tet"])
    assert np.array_equal(got["tet"].cpu().numpy(), ref["tet"])
    assert np.array_equal(got["mask"].cpu().numpy(), ref["mask"])
    assert np.array_equal(got["feat"].cpu().numpy().view(np.uint32), ref["feat"].view(np.uint32))
    # both FP64; the two clippers round differently on slivers (cut parameters near
    # 0 or 1 amplify rounding by the sliver's aspect), the oracle's own partition
    # of unity holds to ~5e-12
    fr = got["frac"].cpu().numpy()
    assert np.max(np.abs(fr - ref["frac"])) <= 1e-10
    assert np.max(np.abs(fr.sum(1) - 1.0)) <= 1e-10


def test_examples_range_and_capacity(psd, orc):
    pos = zeldovich_positions(12, 2.0, seed=62)
    nc = 3
    first, count = 100, 700
    ref = orc.surrogate_examples(pos, nc, first=first, count=count)
    keep = np.array([bin(int(m)).count("1") >= 2 for m in ref["mask"]], dtype=bool)
    got = psd.surrogate_examples(_dev(pos), nc, first_cube=first, n_cubes=count, capacity=50)
    assert got["found"] == int(keep.sum())
    assert np.array_equal(got["tet"].cpu().numpy(), ref["tet"][keep][:50])
    empty = psd.surrogate_examples(_dev(pos), nc, first_cube=5, n_cubes=0)
    assert empty["found"] == 0


def test_examples_mid_plane_closed_form(psd):
    # cube corners at 0.75 + 0.5 i cells: cubes with even index straddle the
    # cell plane at their mid-plane; fractions are C(3,K)/8 sums (see the oracle pins)
    npart, nc = 8, 4
    q = np.moveaxis(np.indices((npart,) * 3, dtype=np.float64), 0, -1)
    pos = np.mod((0.75 + 0.5 * q) / nc, 1.0).astype(np.float32)
    got = psd.surrogate_examples(_dev(pos), nc, min_cells=8)
    fr = got["frac"].cpu().numpy()
    # every cube straddling all three planes: each tet's non-zero fractions are 1/8, 3/8, 3/8, 1/8
    assert got["found"] == 6 * (npart // 2) ** 3
    for row in fr:
        nz = np.sort(row[row > 0])
        assert np.allclose(nz, [1 / 8, 1 / 8, 3 / 8, 3 / 8], rtol=0, atol=1e-14)


def _batch(orc, n_min=300, seed=63):
    pos = zeldovich_positions(16, 2.0, seed=seed)
    ex = orc.surrogate_examples(pos, 4)
    keep = np.array([bin(int(m)).count("1") >= 2 for m in ex["mask"]], dtype=bool)
    ex = {k: v[keep] for k, v in ex.items()}
    assert len(ex["tet"]) >= n_min
    return ex


@pytest.mark.parametrize("scale", [1.0, 3.0])
def test_forward_matches_reference(psd, orc, scale):
    ex = _batch(orc)
    n = 1000 + 37  # several 64-sample tiles and a ragged tail
    x, m = ex["feat"][:n], ex["mask"][:n]
    w = _theta(seed=5, scale=scale)
    got = psd.surrogate_forward(_dev(w), _dev(x), _dev(m)).cpu().numpy()
    ref, _ = S.forward(S.effective(w), x, m)
    mb = S.mask_bits(m)
    assert np.all(got[~mb] == 0.0)
    assert np.allclose(got.sum(1), 1.0, atol=1e-6)
    print(f"forward scale {scale}: relative norm {_rel(got, ref):.3e}, "
          f"max |dp| {np.abs(got - ref).max():.3e}", flush=True)
    assert _rel(got, ref) <= NET_TOL, _rel(got, ref)


def test_backward_matches_reference(psd, orc):
    ex = _batch(orc)
    w = _theta(seed=7)
    rng = np.random.default_rng(8)
    idx = rng.choice(len(ex["tet"]), size=777, replace=False).astype(np.int64)
    g, loss = psd.surrogate_backward(_dev(w), _dev(ex["feat"]), _dev(ex["frac"]), _dev(ex["mask"]),
                                     idx=_dev(idx))
    L, gref = S.backward(S.effective(w), ex["feat"][idx], ex["frac"][idx], ex["mask"][idx])
    g = g.cpu().numpy()
    print(f"backward: loss rel {abs(float(loss.item()) - L) / abs(L):.3e}, "
          f"gradient relative norm {_rel(g, gref):.3e}", flush=True)
    assert float(loss.item()) == pytest.approx(L, rel=5e-3)
    assert _rel(g, gref) <= NET_TOL, _rel(g, gref)
    # every parameter block on its own
    o = 0
    for name, shape in S.LAYOUT:
        k = int(np.prod(shape))
        print(f"  {name}: {_rel(g[o:o + k], gref[o:o + k]):.3e}", flush=True)
        assert _rel(g[o:o + k], gref[o:o + k]) <= NET_TOL, (name, _rel(g[o:o + k], gref[o:o + k]))
        o += k


@pytest.mark.parametrize("batch,n,per_launch,tol", [(64, 64 * 5, 5, (1e-6, 1e-8)),
                                                    (256, 1000, 3, (1e-4, 2e-5))])
def test_train_steps_match_per_step_calls(psd, orc, batch, n, per_launch, tol):
    """Several steps per cooperative launch against one backward and one Adam launch per
    step (each pinned to the FP64 reference above), from the same start and sample order.
    One workgroup (batch 64) adds its gradient in a fixed order, so the two agree to FP32
    rounding; with four the order of the gradient sums varies between runs.  The second
    case has a ragged last batch and splits its 4 steps over two launches (3 + 1)."""
    ex = _batch(orc)
    rng = np.random.default_rng(31)
    order = rng.integers(0, len(ex["tet"]), size=n).astype(np.int64)
    feat, frac, mask = _dev(ex["feat"]), _dev(ex["frac"]), _dev(ex["mask"])
    w0 = _theta(seed=13)
    runs = []
    for spl in (0, per_launch):
        w = _dev(w0)
        st = psd.train_surrogate(w, feat, frac, mask, order, batch=batch, lr=2e-3, lr_final=1e-3,
                                 steps_per_launch=spl)
        torch.cuda.synchronize()
        runs.append((w.cpu().numpy(), st["m"].cpu().numpy(), st["v"].cpu().numpy(),
                     st["losses"].cpu().numpy(), st["step"]))
    (w1, m1, v1, l1, s1), (w2, m2, v2, l2, s2) = runs
    rtol, atol = tol
    steps = (n + batch - 1) // batch
    assert s1 == s2 == steps and len(l1) == len(l2) == steps
    print(f"train steps: max |dw| {np.abs(w1 - w2).max():.3e}, losses {l1} vs {l2}", flush=True)
    assert np.all(np.isfinite(w2)) and np.abs(w2 - w0).max() > 1e-4  # the parameters moved
    assert np.allclose(l2, l1, rtol=max(rtol, 1e-7), atol=0.0)
    assert np.allclose(w2, w1, rtol=rtol, atol=atol)
    assert np.allclose(m2, m1, rtol=rtol, atol=atol)
    assert np.allclose(v2, v1, rtol=rtol, atol=atol * atol)


def test_adam_matches_reference(psd):
    rng = np.random.default_rng(9)
    w = rng.normal(size=S.N_PARAMS).astype(np.float32)
    grads = rng.normal(size=(3, S.N_PARAMS)).astype(np.float32)
    wd, md, vd = _dev(w), torch.zeros(S.N_PARAMS, device="cuda:0"), torch.zeros(S.N_PARAMS, device="cuda:0")
    wr, mr, vr = w.astype(np.float64), np.zeros(S.N_PARAMS), np.zeros(S.N_PARAMS)
    for t in range(3):
        psd.surrogate_adam(wd, _dev(grads[t]), md, vd, t + 1, lr=1e-2)
        wr, mr, vr = S.adam(wr, grads[t].astype(np.float64), mr, vr, t + 1, lr=1e-2)
    assert np.allclose(wd.cpu().numpy(), wr, rtol=1e-5, atol=1e-6)


def _composed_reference(orc, pos, nc, w):
    """Oracle composition: exact deposit, with the eligible tetrahedra's exact fractions
    replaced by the FP64 reference network's probabilities."""
    exact, cnt = orc.deposit_uniform(pos, nc)
    ex = orc.surrogate_examples(pos, nc)
    keep = np.array([bin(int(m)).count("1") >= 2 for m in ex["mask"]], dtype=bool)
    ex = {k: v[keep] for k, v in ex.items()}
    m = 1.0 / (6 * pos.shape[0] * pos.shape[1] * pos.shape[2])
    p, _ = S.forward(S.effective(w), ex["feat"], ex["mask"])
    out = exact.copy()
    for c in range(8):
        d = np.array([(c >> 2) & 1, (c >> 1) & 1, c & 1])
        cell = (ex["lo"] + d) % nc
        np.add.at(out, (cell[:, 0], cell[:, 1], cell[:, 2]), m * (p[:, c] - ex["frac"][:, c]))
    return out, exact, len(ex["tet"]), cnt


@pytest.mark.parametrize("fp64", [False, True])
def test_surrogate_deposit_matches_composition(psd, orc, fp64):
    pos = zeldovich_positions(24, 2.0, seed=64)
    nc = 6
    w = _theta(seed=11)
    ref, exact, n_el, cnt = _composed_reference(orc, pos, nc, w)
    flags = psd.PSD_SURROGATE | (psd.PSD_PREC_FP64 if fp64 else 0)
    ms = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    st = torch.zeros(8, dtype=torch.int64, device="cuda:0")
    got = psd.deposit_uniform(_dev(pos), nc, flags=flags, mass_sum=ms, stats=st,
                              surrogate=_dev(w)).double().cpu().numpy()
    st = st.cpu().numpy()
    assert st[6] == n_el and st[0] == cnt["n_tet"]
    assert st[4] == cnt["n_inverted"] and st[5] == cnt["n_degenerate"]
    assert abs(float(ms.item()) - 1.0) <= 1e-12
    assert abs(got.sum() - 1.0) <= (1e-12 if fp64 else 1e-5)
    # the network's share of the grid is held to the network tolerance
    moved = np.abs(ref - exact).sum()
    assert np.abs(got - ref).sum() <= NET_TOL * moved + 1e-5 * np.abs(ref).sum()


def test_surrogate_flag_needs_parameters(psd):
    pos = zeldovich_positions(4, 0.5, seed=65)
    with pytest.raises(psd.PsdError):
        psd.deposit_uniform(_dev(pos), 4, flags=psd.PSD_SURROGATE)
    with pytest.raises(psd.PsdError):
        psd.deposit_uniform(_dev(pos), 4, flags=psd.PSD_SURROGATE | psd.PSD_METHOD_CELL,
                            surrogate=_dev(_theta()))


def test_training_gains_over_untrained_and_bbox_baseline(psd, orc):
    """Train on GPU-made examples from fresh seeds (GPU kernels end to end), evaluate
    on held-out examples labelled by the oracle."""
    from paper_1612_09491_amd import train as T
    dev = torch.device("cuda:0")
    parts = []
    for k in range(3):
        pos = _dev(zeldovich_positions(48, 2.0, seed=TRAIN_SEED0 + 100 + k))
        ex = psd.surrogate_examples(pos, 12, with_ids=False)
        parts.append(ex)
    ex = {k: torch.cat([p[k] for p in parts]) for k in ("feat", "frac", "mask")}
    n_train = int(ex["mask"].numel())
    print(f"{n_train} training examples")
    pos_ev = zeldovich_positions(32, 2.0, seed=66)
    nc_ev = 8
    ev = orc.surrogate_examples(pos_ev, nc_ev)
    keep = np.array([bin(int(m)).count("1") >= 2 for m in ev["mask"]], dtype=bool)
    ev = {k: v[keep] for k, v in ev.items()}
    w = torch.from_numpy(T.initial_parameters(3)).to(dev)

    def frac_l1(params):
        p = psd.surrogate_forward(params, _dev(ev["feat"]), _dev(ev["mask"])).cpu().numpy()
        return float(np.abs(p - ev["frac"]).sum(1).mean())

    l1_untrained = frac_l1(w)
    l1_bbox = float(np.abs(S.bbox_overlap_fractions(ev["feat"], ev["mask"]) - ev["frac"]).sum(1).mean())
    rec = T.train(w, ex, epochs=4, batch=2048, lr=3e-3, lr_final=1e-4, seed=4, log=print)
    l1_trained = frac_l1(w)
    print(f"fraction L1: untrained {l1_untrained:.4f} bbox {l1_bbox:.4f} trained {l1_trained:.4f} "
          f"({rec['seconds']:.1f} s, {rec['steps']} steps, losses {rec['epoch_loss']})")
    assert rec["epoch_loss"][-1] < rec["epoch_loss"][0]
    assert l1_trained < 0.5 * l1_bbox and l1_trained < 0.25 * l1_untrained
    # the same gain on the deposited density of the held-out box
    exact, _ = orc.deposit_uniform(pos_ev, nc_ev)
    got = psd.deposit_uniform(_dev(pos_ev), nc_ev, flags=psd.PSD_SURROGATE | psd.PSD_PREC_FP64,
                              surrogate=w).cpu().numpy()
    base = exact.copy()
    m = 1.0 / (6 * 32 ** 3)
    bb = S.bbox_overlap_fractions(ev["feat"], ev["mask"])
    for c in range(8):
        d = np.array([(c >> 2) & 1, (c >> 1) & 1, c & 1])
        cell = (ev["lo"] + d) % nc_ev
        np.add.at(base, (cell[:, 0], cell[:, 1], cell[:, 2]), m * (bb[:, c] - ev["frac"][:, c]))
    l1_dens = float(np.abs(got - exact).sum() / exact.sum())
    l1_dens_bbox = float(np.abs(base - exact).sum() / exact.sum())
    print(f"density L1: surrogate {l1_dens:.3e} bbox baseline {l1_dens_bbox:.3e}")
    assert l1_dens < 0.5 * l1_dens_bbox


def _oracle_fractions(orc, tets):
    """|T cap C_c| / |T| for the 8 cells of the block by the oracle's clipper."""
    out = np.zeros((len(tets), 8))
    for i, v in enumerate(tets.astype(np.float64)):
        e = v[1:] - v[0]
        vol = abs(np.linalg.det(e)) / 6.0
        for c in range(8):
            lo = np.array([(c >> 2) & 1, (c >> 1) & 1, c & 1], dtype=np.float64)
            out[i, c] = orc.clip_tet_box(v, lo, lo + 1.0) / vol
    return out


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build_oracle(force=False)
    return oracle


def test_exact_fractions_match_oracle(psd, orc):
    rng = np.random.default_rng(21)
    big = rng.uniform(0.0, 2.0, (300, 4, 3))                      # up to all 8 cells
    centre = rng.uniform(0.3, 1.7, (300, 1, 3))
    small = centre + rng.normal(scale=0.25, size=(300, 4, 3))      # 1..8 cells
    small = np.clip(small, 0.0, 1.999)
    inside = rng.uniform(1.05, 1.95, (100, 4, 3))                  # one cell
    base = rng.uniform(0.1, 1.9, (100, 3, 3))                      # slivers
    w = rng.dirichlet([1, 1, 1], size=100)
    sliver = np.concatenate([base, (np.einsum("nk,nkd->nd", w, base) +
                                    rng.normal(scale=1e-3, size=(100, 3)))[:, None]], axis=1)
    sliver = np.clip(sliver, 0.0, 1.999)
    tets = np.concatenate([big, small, inside, sliver]).astype(np.float32)
    got = psd.exact_fractions(torch.from_numpy(tets).cuda()).cpu().numpy()
    ref = _oracle_fractions(orc, tets)
    assert np.abs(got - ref).max() <= 1e-10
    assert np.abs(got.sum(axis=1) - 1.0).max() <= 1e-12
    # a tetrahedron inside one cell puts everything there
    cell = (4 * (inside[:, 0, 0] >= 1) + 2 * (inside[:, 0, 1] >= 1) + (inside[:, 0, 2] >= 1)).astype(int)
    assert np.array_equal(np.argmax(got[600:700], axis=1), cell)


def test_exact_fractions_degenerate_and_outside(psd):
    t = np.zeros((5, 4, 3), dtype=np.float32)
    # zero volume (a repeated vertex): all in the centroid's cell (1, 0, 1) -> c = 5
    t[0] = [[1.2, 0.3, 1.5], [1.6, 0.2, 1.1], [1.2, 0.3, 1.5], [1.4, 0.9, 1.3]]
    t[1] = [[0.2, 0.3, 0.5], [2.0, 0.2, 0.1], [0.2, 0.9, 0.5], [0.4, 0.9, 0.3]]  # x = 2 is outside
    t[2] = [[0.2, 0.3, 0.5], [0.6, 0.2, 0.1], [0.2, 0.9, 0.5], [-0.1, 0.9, 0.3]]
    t[3] = [[0.2, 0.3, 0.5], [0.6, 0.2, np.nan], [0.2, 0.9, 0.5], [0.4, 0.9, 0.3]]
    t[4] = [[0.2, 0.3, 0.5], [1.6, 0.2, 0.1], [0.2, 1.9, 0.5], [0.4, 0.9, 1.3]]
    got = psd.exact_fractions(torch.from_numpy(t).cuda()).cpu().numpy()
    assert np.array_equal(got[0], np.eye(8)[5])
    assert np.isnan(got[1:4]).all()
    assert np.isfinite(got[4]).all() and abs(got[4].sum() - 1.0) <= 1e-12
    empty = psd.exact_fractions(torch.zeros((0, 4, 3), dtype=torch.float32, device="cuda"))
    assert empty.shape == (0, 8)
