"""Pins of the FP64 surrogate reference and of the oracle's surrogate examples.

The network reference is checked against an independent implementation of
the same function (PyTorch CPU, float64, autograd), against central finite
differences, and against PyTorch's Adam.  The examples (eligibility, features,
exact overlap fractions) are checked against closed forms from the order
statistics of three uniform variables, which give the overlap fractions of a
split tetrahedron whose cube straddles cell planes at its mid-planes.
"""

import math

import numpy as np
import pytest
import torch

from oracle import surrogate as S
from synth import lattice_positions, uniform_segments, zeldovich_positions


def _theta(seed=3, scale=1.0):
    segs = []
    for name, shape in S.LAYOUT:
        fan_in = shape[1] if len(shape) == 2 else S.LAYOUT[[n for n, _ in S.LAYOUT].index(
            "W" + name[1:])][1][1]
        segs.append((int(np.prod(shape)), scale / math.sqrt(fan_in)))
    return uniform_segments(segs, seed)


def _batch(n=37, seed=4):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 2.0, size=(n, 12)).astype(np.float32)
    # bbox masks: the cells d <= span of per-axis spans in {0, 1}
    span = rng.integers(0, 2, size=(n, 3))
    span[:4] = [[0, 0, 0], [0, 1, 1], [1, 0, 1], [1, 1, 1]]
    mask = np.zeros(n, dtype=np.uint8)
    for c in range(8):
        d = np.array([(c >> 2) & 1, (c >> 1) & 1, c & 1])
        mask |= (np.all(d[None, :] <= span, axis=1).astype(np.uint8) << c)
    mb = S.mask_bits(mask)
    y = np.where(mb, rng.uniform(size=(n, 8)), 0.0)
    y /= y.sum(1, keepdims=True)
    return x, mask, y


def test_layout_size():
    assert S.N_PARAMS == 9672


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(0)
    a = rng.normal(scale=3.0, size=4096).astype(np.float32)
    # exact ties: low 16 bits = 0x8000, both parities of the kept bit
    ties = (np.arange(1, 257, dtype=np.uint32) << 16 | 0x3F800000 | 0x8000).view(np.float32)
    a = np.concatenate([a, ties, -ties, np.float32([0.0, -0.0, 1.0, 65504.0])])
    want = torch.from_numpy(a).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(S.bf16_round(a).view(np.uint32), want.view(np.uint32))


def _torch_net(theta):
    P = S.unpack(theta)
    layers = []
    for k in range(1, 5):
        lin = torch.nn.Linear(P[f"W{k}"].shape[1], P[f"W{k}"].shape[0]).double()
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(P[f"W{k}"]))
            lin.bias.copy_(torch.from_numpy(P[f"b{k}"]))
        layers.append(lin)
        if k < 4:
            layers.append(torch.nn.SiLU())
    return torch.nn.Sequential(*layers)


def _torch_loss(net, x, y, mask):
    z = net(torch.from_numpy(x.astype(np.float64)))
    mb = torch.from_numpy(S.mask_bits(mask))
    lp = torch.log_softmax(z.masked_fill(~mb, -math.inf), dim=1)
    lp = lp.masked_fill(~mb, 0.0)
    return -(torch.from_numpy(y) * lp).sum() / x.shape[0], lp


def test_forward_matches_torch():
    theta = S.effective(_theta())
    x, mask, y = _batch()
    p, _ = S.forward(theta, x, mask)
    xc, r = S.canonical(x, mask)
    net = _torch_net(theta)
    L, lp = _torch_loss(net, xc, S.to_canonical_cells(y, r), mask)
    pt = torch.exp(lp).masked_fill(~torch.from_numpy(S.mask_bits(mask)), 0.0).detach().numpy()
    assert np.allclose(p, S.from_canonical_cells(pt, r), rtol=1e-12, atol=1e-15)
    assert S.loss(theta, x, y, mask) == pytest.approx(float(L.detach()), rel=1e-12)


def test_softmax_is_a_distribution_on_the_mask():
    theta = S.effective(_theta(scale=4.0))
    x, mask, _ = _batch(200)
    p, _ = S.forward(theta, x, mask)
    mb = S.mask_bits(mask)
    assert np.all(p[~mb] == 0.0)
    assert np.all(p[mb] > 0.0)
    assert np.allclose(p.sum(1), 1.0, rtol=0, atol=1e-15)
    single = mask == 1
    assert np.all(p[single, 0] == 1.0)


def test_backward_matches_torch_autograd():
    theta = S.effective(_theta())
    x, mask, y = _batch()
    L, g = S.backward(theta, x, y, mask)
    net = _torch_net(theta)
    xc, r = S.canonical(x, mask)
    Lt, _ = _torch_loss(net, xc, S.to_canonical_cells(y, r), mask)
    Lt.backward()
    gt = {}
    for k, idx in zip(range(1, 5), (0, 2, 4, 6)):
        gt[f"W{k}"] = net[idx].weight.grad.numpy()
        gt[f"b{k}"] = net[idx].bias.grad.numpy()
    assert L == pytest.approx(float(Lt.detach()), rel=1e-12)
    assert np.allclose(g, S.pack(gt), rtol=1e-10, atol=1e-14)


def test_backward_central_differences():
    theta = S.effective(_theta())
    x, mask, y = _batch(29, seed=9)
    _, g = S.backward(theta, x, y, mask)
    rng = np.random.default_rng(5)
    # a few coordinates of every parameter block
    idx, o = [], 0
    for _, shape in S.LAYOUT:
        n = int(np.prod(shape))
        idx += list(o + rng.choice(n, size=min(n, 8), replace=False))
        o += n
    h = 1e-6
    fd = []
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd.append((S.loss(tp, x, y, mask) - S.loss(tm, x, y, mask)) / (2 * h))
    fd = np.array(fd)
    assert np.linalg.norm(fd - g[idx]) <= 1e-6 * np.linalg.norm(g[idx])


def _dyadic_tets(n=300, seed=12):
    """Tetrahedra with coordinates k/64 in [0, 2) and the mask of their bbox cells."""
    rng = np.random.default_rng(seed)
    x = (rng.integers(0, 128, size=(n, 12)) / 64.0).astype(np.float32)
    v = x.reshape(n, 4, 3)
    lo = np.floor(v.min(1))
    x = (v - lo[:, None, :]).reshape(n, 12).astype(np.float32)
    span = (np.floor(v.max(1)) - lo).astype(int)
    mask = np.zeros(n, dtype=np.uint8)
    for c in range(8):
        d = np.array([(c >> 2) & 1, (c >> 1) & 1, c & 1])
        mask |= (np.all(d[None, :] <= span, axis=1).astype(np.uint8) << c)
    return x, mask


def test_canonical_pose_ignores_vertex_order():
    x, mask = _dyadic_tets()
    xc, r = S.canonical(x, mask)
    for perm in __import__("itertools").permutations(range(4)):
        xp = x.reshape(-1, 4, 3)[:, list(perm), :].reshape(-1, 12)
        xq, rq = S.canonical(xp, mask)
        assert np.array_equal(xq, xc) and np.array_equal(rq, r)
    # sorted vertices, reflections only on straddling axes, centroid at or below the plane
    v = xc.reshape(-1, 4, 3)
    # coordinates are k/64 with k < 128: an exact lexicographic key in base 128
    keys = (v[:, :, 0] * 64).astype(np.int64) * 16384 + (v[:, :, 1] * 64).astype(np.int64) * 128 + \
        (v[:, :, 2] * 64).astype(np.int64)
    assert np.all(np.diff(keys, axis=1) >= 0)
    for a, bit in enumerate(S.AXIS_BIT):
        straddle = (mask >> bit) & 1 == 1
        assert np.all((r & bit)[~straddle] == 0)
        assert np.all(v[straddle, :, a].astype(np.float64).sum(1) <= 4.0)


def test_canonical_reflection_swaps_cells():
    x, mask = _dyadic_tets(seed=13)
    theta = S.effective(_theta())
    p, _ = S.forward(theta, x, mask)
    v = x.reshape(-1, 4, 3).astype(np.float64)
    for bits in range(1, 8):
        flip = np.array([(bits >> 2) & 1, (bits >> 1) & 1, bits & 1], dtype=bool)
        straddle = np.stack([(mask >> b) & 1 == 1 for b in S.AXIS_BIT], 1)
        ok = np.all(straddle | ~flip[None, :], axis=1)  # only reflect straddling axes
        # and avoid ties at the middle plane, where either pose is canonical
        sums = v.sum(1)
        ok &= np.all(~flip[None, :] | (sums != 4.0), axis=1)
        vr = np.where(flip[None, None, :], 2.0 - v, v).astype(np.float32).reshape(-1, 12)
        xc, r = S.canonical(x[ok], mask[ok])
        xq, rq = S.canonical(vr[ok], mask[ok])
        assert np.array_equal(xq, xc) and np.array_equal(rq, r ^ bits)
        pr, _ = S.forward(theta, vr[ok], mask[ok])
        want = np.take_along_axis(p[ok], np.arange(8)[None, :] ^ bits, 1)
        # same network inputs; only the matrix products' blocking differs with the batch
        assert np.allclose(pr, want, rtol=1e-13, atol=1e-16), bits


def test_adam_matches_torch():
    rng = np.random.default_rng(6)
    w = rng.normal(size=50)
    grads = rng.normal(size=(3, 50))
    wt = torch.tensor(w.copy(), requires_grad=True)
    opt = torch.optim.Adam([wt], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(50)
    v = np.zeros(50)
    for t in range(3):
        w, m, v = S.adam(w, grads[t], m, v, t + 1, lr=1e-2)
        wt.grad = torch.from_numpy(grads[t].copy())
        opt.step()
    assert np.allclose(w, wt.detach().numpy(), rtol=1e-14, atol=1e-15)


# --- examples --------------------------------------------------------------


def _order_stat_fraction(perm, straddle, high):
    """Share of {1 >= u_perm0 >= u_perm1 >= u_perm2 >= 0} with u_a > 1/2 exactly for the
    straddling axes a with high[a].  The ordered triple is distributed as the order
    statistics of three iid U(0,1); the rank-r value exceeds 1/2 iff at least r+1 of
    the three samples do, and K samples exceed 1/2 with probability C(3,K)/8."""
    rank = {a: r for r, a in enumerate(perm)}
    tot = 0.0
    for K in range(4):
        ok = all((K >= rank[a] + 1) == bool(high[a]) for a in range(3) if straddle[a])
        if ok:
            tot += math.comb(3, K) / 8.0
    return tot


PERMS = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]


def test_examples_mid_plane_straddle_closed_form(orc):
    # lattice at 0.75 + 0.5 i cells: even cubes straddle a cell plane at their
    # mid-plane, odd cubes lie inside one cell (per axis)
    npart, nc = 8, 4
    q = np.moveaxis(np.indices((npart,) * 3, dtype=np.float64), 0, -1)
    pos = np.mod((0.75 + 0.5 * q) / nc, 1.0).astype(np.float32)
    ex = orc.surrogate_examples(pos, nc, compact=False)
    assert ex["flag"].all()
    n_checked = 0
    for t in range(6 * npart ** 3):
        cube, p = divmod(t, 6)
        ijk = np.unravel_index(cube, (npart,) * 3)
        straddle = [ijk[a] % 2 == 0 for a in range(3)]
        want_mask = 0
        want = np.zeros(8)
        for c in range(8):
            d = [(c >> 2) & 1, (c >> 1) & 1, c & 1]
            if any(d[a] and not straddle[a] for a in range(3)):
                continue
            want_mask |= 1 << c
            want[c] = _order_stat_fraction(PERMS[p], straddle, d)
        assert ex["mask"][t] == want_mask
        assert np.allclose(ex["frac"][t], want, rtol=0, atol=1e-14), (t, ex["frac"][t], want)
        # features: vertex minus bbox origin, cube-local offsets plus 0.25 or 0.75
        f = ex["feat"][t].reshape(4, 3)
        base = np.array([0.75 if s else 0.25 for s in straddle])
        assert np.allclose(f.min(0), base) and np.allclose(f.max(0), base + 0.5)
        n_checked += 1
    assert n_checked == 6 * 512


def test_examples_touching_cells_get_zero(orc):
    # lattice at 0.5 i cells: odd cubes end exactly on a cell plane, so their
    # bbox spans 2 cells per axis but all the volume is in the lower one
    npart, nc = 8, 4
    pos = lattice_positions(npart)
    ex = orc.surrogate_examples(pos, nc, compact=False)
    assert ex["flag"].all()
    assert np.array_equal(ex["frac"][:, 0], np.ones(6 * npart ** 3))
    assert np.all(ex["frac"][:, 1:] == 0.0)


def test_examples_random_partition_and_eligibility(orc):
    pos = zeldovich_positions(12, 2.0, seed=51)
    nc = 3
    ex = orc.surrogate_examples(pos, nc, compact=False)
    fl = ex["flag"].astype(bool)
    assert 0.4 < fl.mean() < 0.95
    mb = S.mask_bits(ex["mask"])
    assert np.all(ex["frac"][~mb] == 0.0)
    assert np.all(ex["frac"][fl] >= -1e-12)
    assert np.allclose(ex["frac"][fl].sum(1), 1.0, rtol=0, atol=1e-10)
    assert np.all((ex["feat"][fl] >= 0.0) & (ex["feat"][fl] <= 2.0))
    # eligibility recomputed from the unwrapped tetrahedra, cube by cube
    for cube in range(0, 12 ** 3, 37):
        i, j, k = np.unravel_index(cube, (12,) * 3)
        tets, det = orc.cube_tets(pos, (nc, nc, nc), i, j, k)
        for p in range(6):
            span = np.floor(tets[p].max(0)) - np.floor(tets[p].min(0))
            assert fl[6 * cube + p] == bool(np.all(span <= 1) and abs(det[p]) > 0)


def test_bbox_baseline_one_hot_and_normalised():
    x = np.array([[0.1, 0.2, 0.3, 0.5, 0.2, 0.3, 0.1, 0.9, 0.3, 0.1, 0.2, 0.8],
                  [0.5, 0.5, 0.5, 1.5, 0.5, 0.5, 0.5, 1.5, 0.5, 0.5, 0.5, 1.5]], dtype=np.float32)
    mask = np.array([1, 0xFF], dtype=np.uint8)
    b = S.bbox_overlap_fractions(x, mask)
    assert b[0, 0] == 1.0 and np.all(b[0, 1:] == 0.0)
    # second box is [0.5,1.5]^3: an eighth in each cell
    assert np.allclose(b[1], 1.0 / 8.0)
