"""Own-work cost model of the cumulative deposit kernel, counted on the CPU.

The default deposit (psd_cumulative.hip) computes, for every column (a, b) of a
tetrahedron's bounding box in its walk frame, the pieces of T cut by the two planes
u <= a+1 and v <= b+1 (Section 6.3's inside-mask splitting, applied twice), spreads
each piece's volume over the cells of the third axis with the exact distribution of
that coordinate over a tetrahedron, and takes 2-D differences of the column sums.
Its work is counted per event:

  tet      a tetrahedron that needs the walk (bbox of 2 cells or more, non-zero volume)
  column   one two-plane column of a tile, halo columns included: the u-split
  xpiece   a piece of the u-split (1 or 3 per column): the v-split
  piece    a piece of the v-split (1 or 3 per x-piece): the z distribution set-up
  level    one z level walked by a piece (one unit-step difference of its cubic)
  colcell  one (column, level) slot of a tile: zeroed in phase 1, differenced in phase 2
  nz       one non-zero cell mass scattered

Unit costs (frozen; lane operations, one add, mul, FMA, compare, select, min/max,
cvt, rcp, LDS access or atomic = 1) are the operations the kernel's source performs
per event, read off the code:

  tet     250  corner loads and scaling, periodic unwrap, determinant, longest edge,
               bbox, walk-frame permutation, relative vertices, planning
  column  137  4 plane distances, the split (mask, 4 cut parameters with one Newton
               step each, 3 fractions, selects) and the cut points' 2 remaining coordinates
  xpiece  110  the second split, with the cut points' last coordinate
  piece   122  sorting 4 heights, 6 differences, the 7 reciprocals of the cubic pieces,
               and the region coefficients of the distribution
  level     6  the quadratic step (2 FMA), its abscissa, the LDS add, loop control
  colcell  15  zeroing, 4 LDS reads, the 2-D difference, the threshold, the output step
  nz        5  scale, convert, atomic, FP64 mass sum

The model prices the kernel's own work (not the paper's per-cell splitting: that is the
oracle's counting mode, reported beside it as an equivalent rate).  ``count_events``
replays the kernel's geometry on a sample of Lagrangian cubes in float64 numpy: the
same unwrap, bbox, walk frame, tiling of large tetrahedra and piece triangulation, so
its counts agree with the kernel's work counters except where rounding decides an
on-plane vertex.  Where a split leaves three vertices inside, the kernel walks the
complement: for y, the x-piece whole and minus its one outside tetrahedron (two pieces
instead of three); for x, when the tile holds the bbox's last row, minus the one outside
tetrahedron (the 2-D differences then add the last row's column back).  This module is
measurement code: it shares no code with the kernels or with the oracle.
"""

from __future__ import annotations

import numpy as np

COST = {"tet": 250, "column": 137, "xpiece": 110, "piece": 122, "level": 6, "colcell": 15,
        "nz": 5}

EVENTS = ("tet", "column", "xpiece", "piece", "level", "colcell")

# Freudenthal split: corner index q = 4a + 2b + c; tetrahedron p has corners
# (0, q1[p], q2[p], 7) for the axis permutations 012, 021, 102, 120, 201, 210.
_Q1 = (4, 4, 2, 2, 1, 1)
_Q2 = (6, 5, 6, 3, 5, 3)


def own_ops(counts: dict) -> float:
    """Lane operations of the counted events (counts per event name, plus "nz")."""
    return float(sum(COST[k] * counts.get(k, 0) for k in COST))


def _tets(pos: np.ndarray, nc, cubes: np.ndarray):
    """Unwrapped vertices (cell units) of the 6 tetrahedra of each listed cube: [n, 4, 3]."""
    n0, n1, n2 = pos.shape[:3]
    nc = np.asarray(nc, dtype=np.float64)
    i = cubes // (n1 * n2)
    j = (cubes // n2) % n1
    k = cubes % n2
    corner = []
    for q in range(8):
        ii = (i + ((q >> 2) & 1)) % n0
        jj = (j + ((q >> 1) & 1)) % n1
        kk = (k + (q & 1)) % n2
        corner.append(pos[ii, jj, kk].astype(np.float64) * nc)   # box = 1
    corner = np.stack(corner, axis=1)                               # [m, 8, 3]
    c0 = corner[:, 0]
    c0w = c0 - nc * np.floor(c0 / nc)
    d = corner - c0[:, None, :]
    d = d - nc * np.rint(d / nc)
    cw = c0w[:, None, :] + d
    cw[:, 0] = c0w
    tets = np.stack([np.stack([cw[:, 0], cw[:, _Q1[p]], cw[:, _Q2[p]], cw[:, 7]], axis=1)
                     for p in range(6)], axis=1)                  # [m, 6, 4, 3]
    return tets.reshape(-1, 4, 3)


def _split(V: np.ndarray, d: np.ndarray):
    """Inside parts (d >= 0) of tetrahedra V [m, 4, k] against plane values d [m, 4], with
    the kernel's triangulation.  Returns (children [c, 4, k], parent index [c])."""
    ins = d >= 0
    nin = ins.sum(axis=1)
    perm = np.argsort(~ins, axis=1, kind="stable")          # inside first, ascending
    P = np.take_along_axis(V, perm[:, :, None], axis=1)
    dp = np.take_along_axis(d, perm, axis=1)

    def cut(x, y):  # point on edge x -> y where the plane value vanishes (x inside)
        den = dp[:, x] - dp[:, y]
        t = np.where(den > 0, dp[:, x] / np.where(den > 0, den, 1.0), 0.0)
        return P[:, x] + t[:, None] * (P[:, y] - P[:, x])

    out, parent = [], []
    idx = np.arange(len(V))
    for n_in in (1, 2, 3, 4):
        sel = nin == n_in
        if not sel.any():
            continue
        if n_in == 4:
            out.append(P[sel])
            parent.append(idx[sel])
            continue
        a = P[sel, 0]
        if n_in == 1:
            out.append(np.stack([a, cut(0, 1)[sel], cut(0, 2)[sel], cut(0, 3)[sel]], axis=1))
            parent.append(idx[sel])
            continue
        if n_in == 2:
            U0, U1, U2 = a, cut(0, 2)[sel], cut(0, 3)[sel]
            W0, W1, W2 = P[sel, 1], cut(1, 2)[sel], cut(1, 3)[sel]
        else:
            U0, U1, U2 = a, P[sel, 1], P[sel, 2]
            W0, W1, W2 = cut(0, 3)[sel], cut(1, 3)[sel], cut(2, 3)[sel]
        for ch in ((U0, U1, U2, W2), (U0, U1, W1, W2), (U0, W0, W1, W2)):
            out.append(np.stack(ch, axis=1))
            parent.append(idx[sel])
    if not out:
        return np.zeros((0,) + V.shape[1:]), np.zeros(0, dtype=np.int64)
    return np.concatenate(out), np.concatenate(parent)


def _tile_shape(ext, cap):
    tl = min(ext[2], cap // 4)
    tb = min(ext[1], cap // (2 * tl) - 1)
    ta = min(ext[0], cap // (tl * (tb + 1)) - 1)
    return ta, tb, tl


def count_events(pos: np.ndarray, nc, cubes: np.ndarray, cap: int = 1024,
                 batch_tets: int = 4000) -> dict:
    """Work events of the cumulative kernel with a `cap`-entry LDS buffer on the
    tetrahedra of the listed Lagrangian cubes (positions float32 [np0, np1, np2, 3],
    periodic unit box, grid nc)."""
    nc3 = np.array([nc] * 3 if np.ndim(nc) == 0 else nc, dtype=np.int64)
    V = _tets(pos, nc3, np.asarray(cubes, dtype=np.int64))
    e = V[:, 1:] - V[:, :1]
    D = np.einsum("ij,ij->i", e[:, 0], np.cross(e[:, 1], e[:, 2]))
    l2 = np.max([((V[:, a] - V[:, b]) ** 2).sum(axis=1) for a in range(4) for b in range(a + 1, 4)],
                axis=0)
    lo = np.floor(V.min(axis=1))
    ext = (np.floor(V.max(axis=1)) - lo + 1).astype(np.int64)
    ncell = ext.prod(axis=1)
    walk = (np.abs(D) > 1e-12 * l2 * np.sqrt(l2)) & (ncell >= 2)
    counts = {k: 0 for k in EVENTS}
    counts["tets_sampled"] = int(len(V))
    counts["tet"] = int(walk.sum())
    V, lo, ext = V[walk], lo[walk], ext[walk]
    # walk frame: the longest bbox side last (ties keep the later grid axis)
    e0, e1, e2 = ext[:, 0], ext[:, 1], ext[:, 2]
    w2 = np.where((e0 > e1) & (e0 > e2), 0, np.where(e1 > e2, 1, 2))
    w0 = np.where(w2 == 0, 1, 0)
    w1 = np.where(w2 == 2, 1, 2)
    axes = np.stack([w0, w1, w2], axis=1)
    vr = np.take_along_axis(V - lo[:, None, :], axes[:, None, :], axis=2)
    ex = np.take_along_axis(ext, axes, axis=1)
    # of the two shorter axes the first split goes along the one with fewer three-piece
    # columns: (floor of the 3rd smallest coordinate - floor of the 2nd) x the other extent
    srt = np.sort(vr[:, :, :2], axis=1)
    rows = np.floor(srt[:, 2]) - np.floor(srt[:, 1])
    swap = rows[:, 1] * ex[:, 0] < rows[:, 0] * ex[:, 1]
    order = np.where(swap[:, None], [1, 0, 2], [0, 1, 2])
    vr = np.take_along_axis(vr, order[:, None, :], axis=2)
    # the kernel keeps each tetrahedron's vertices in increasing walk-frame x
    # (ties by vertex index), which fixes the triangulation of its pieces
    vr = np.take_along_axis(vr, np.argsort(vr[:, :, 0], axis=1, kind="stable")[:, :, None], axis=1)
    ex = np.take_along_axis(ex, order, axis=1)
    for s in range(0, len(vr), batch_tets):
        _count_batch(vr[s:s + batch_tets], ex[s:s + batch_tets], cap, counts)
    return counts


def _count_batch(vr, ex, cap, counts):
    # columns of every tile: (tet, a, b, l0, tl, halo)
    T, A, B, L0, TL, HALO, LAST = [], [], [], [], [], [], []
    for t in range(len(vr)):
        e = [int(x) for x in ex[t]]
        if e[0] * e[1] * e[2] <= cap:
            tiles = [(0, e[0], 0, e[1], 0, e[2])]
        else:
            ta, tb, tl = _tile_shape(e, cap)
            tiles = [(a0, min(ta, e[0] - a0), b0, min(tb, e[1] - b0), l0, min(tl, e[2] - l0))
                     for l0 in range(0, e[2], tl) for b0 in range(0, e[1], tb)
                     for a0 in range(0, e[0], ta)]
        for a0, ta, b0, tb, l0, tl in tiles:
            ha, hb = (1 if a0 > 0 else 0), (1 if b0 > 0 else 0)
            aa, bb = np.meshgrid(np.arange(a0 - ha, a0 + ta), np.arange(b0 - hb, b0 + tb),
                                 indexing="ij")
            n = aa.size
            T.append(np.full(n, t))
            A.append(aa.ravel())
            B.append(bb.ravel())
            L0.append(np.full(n, l0))
            TL.append(np.full(n, tl))
            HALO.append(((aa < a0) | (bb < b0)).ravel())
            LAST.append(np.full(n, a0 + ta == e[0]))
    T, A, B = np.concatenate(T), np.concatenate(A), np.concatenate(B)
    L0, TL, HALO = np.concatenate(L0), np.concatenate(TL), np.concatenate(HALO)
    LAST = np.concatenate(LAST)
    counts["column"] += int(T.size)
    counts["colcell"] += int(TL.sum())
    verts = vr[T]                                           # [c, 4, 3]
    X = (A + 1).astype(np.float64)
    cx = (A + 1) < ex[T, 0]
    dx = np.where(cx[:, None], X[:, None] - verts[:, :, 0], 1.0)
    # the x complement: three vertices inside x <= a+1 (vertices in increasing x)
    # and the tile holding the bbox's last row -> the one outside tetrahedron
    cmp = cx & (dx[:, 2] >= 0) & (dx[:, 3] < 0) & LAST
    Pa, para = _split(verts[~cmp][:, :, 1:], dx[~cmp])
    vc = verts[cmp]
    d3 = vc[:, 3, 0] - X[cmp]
    pts = [vc[:, 3]]
    for q in range(3):
        t = d3 / (d3 - (vc[:, q, 0] - X[cmp]))
        pts.append(vc[:, 3] + t[:, None] * (vc[:, q] - vc[:, 3]))
    P1 = np.concatenate([Pa, np.stack(pts, axis=1)[:, :, 1:]])
    par1 = np.concatenate([np.flatnonzero(~cmp)[para], np.flatnonzero(cmp)])
    counts["xpiece"] += int(len(P1))
    Y = (B[par1] + 1).astype(np.float64)
    cy = (B[par1] + 1) < ex[T[par1], 1]
    dy = np.where(cy[:, None], Y[:, None] - P1[:, :, 0], 1.0)
    # the y complement: three vertices inside y <= b+1 -> the x-piece whole and its
    # one outside tetrahedron (cut points from the inside vertices toward it)
    three = (dy >= 0).sum(axis=1) == 3
    Pb, parb = _split(P1[~three][:, :, 1:], dy[~three])
    Q = P1[three]
    dq = dy[three]
    perm = np.argsort(dq < 0, axis=1, kind="stable")     # inside first, then the outside one
    Qp = np.take_along_axis(Q, perm[:, :, None], axis=1)
    dp = np.take_along_axis(dq, perm, axis=1)
    out = [Qp[:, 3]]
    for q in range(3):
        t = dp[:, q] / (dp[:, q] - dp[:, 3])
        out.append(Qp[:, q] + t[:, None] * (Qp[:, 3] - Qp[:, q]))
    idx3 = np.flatnonzero(three)
    P2 = np.concatenate([Pb, Q[:, :, 1:], np.stack(out, axis=1)[:, :, 1:]])
    par2 = np.concatenate([np.flatnonzero(~three)[parb], idx3, idx3])
    counts["piece"] += int(len(P2))
    col = par1[par2]
    z = P2[:, :, 0]
    lA = np.maximum(np.floor(z.min(axis=1)), L0[col])
    lB = np.minimum(np.floor(z.max(axis=1)), L0[col] + TL[col] - 1)
    counts["level"] += int(np.maximum(lB - lA + 1, 0).sum())
