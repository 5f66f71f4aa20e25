"""Exact-rational volume of a tetrahedron clipped by an axis-aligned box.

Independent brute force used to pin the oracle's clipper: the intersection is
the polytope {x : a_i . x <= b_i} of 4 tetrahedron and 6 box half-spaces.
Its vertices are enumerated from every triple of planes (Cramer's rule in
``fractions.Fraction``), and its volume is the sum over facets of the fan
tetrahedra to an interior point.  Everything is exact for rational inputs.
"""

from __future__ import annotations

import functools
import itertools
from fractions import Fraction as Fr


def _sub(a, b):
    return (a[0] - b[0], a[1] - b[1], a[2] - b[2])


def _dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def _cross(a, b):
    return (a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0])


def _det(a, b, c):
    return _dot(a, _cross(b, c))


def tet_halfspaces(v):
    """Outward half-spaces (a, b), a.x <= b, of a non-degenerate tetrahedron."""
    v = [tuple(Fr(x) for x in p) for p in v]
    hs = []
    for l in range(4):
        i, j, k = [m for m in range(4) if m != l]
        n = _cross(_sub(v[j], v[i]), _sub(v[k], v[i]))
        if _dot(n, _sub(v[l], v[i])) > 0:
            n = (-n[0], -n[1], -n[2])
        hs.append((n, _dot(n, v[i])))
    return hs


def box_halfspaces(lo, hi):
    hs = []
    for k in range(3):
        e = [Fr(0)] * 3
        e[k] = Fr(1)
        hs.append((tuple(e), Fr(hi[k])))
        e = [Fr(0)] * 3
        e[k] = Fr(-1)
        hs.append((tuple(e), Fr(-lo[k])))
    return hs


def _solve3(rows, rhs):
    d = _det(rows[0], rows[1], rows[2])
    if d == 0:
        return None
    # Cramer's rule on the transposed system
    cols = list(zip(*rows))
    out = []
    for k in range(3):
        c = [list(col) for col in cols]
        c[k] = list(rhs)
        out.append(_det(tuple(c[0]), tuple(c[1]), tuple(c[2])) / d)
    return tuple(out)


def polytope_volume(halfspaces) -> Fr:
    verts = set()
    for (a1, b1), (a2, b2), (a3, b3) in itertools.combinations(halfspaces, 3):
        x = _solve3([a1, a2, a3], [b1, b2, b3])
        if x is None:
            continue
        if all(_dot(a, x) <= b for a, b in halfspaces):
            verts.add(x)
    if len(verts) < 4:
        return Fr(0)
    verts = list(verts)
    n = len(verts)
    c = tuple(sum(p[k] for p in verts) / n for k in range(3))
    vol = Fr(0)
    for a, b in halfspaces:
        on = [p for p in verts if _dot(a, p) == b]
        if len(on) < 3:
            continue
        drop = max(range(3), key=lambda k: abs(a[k]))
        keep = [k for k in range(3) if k != drop]
        fc = tuple(sum(p[k] for p in on) / len(on) for k in range(3))

        def rel(p):
            return (p[keep[0]] - fc[keep[0]], p[keep[1]] - fc[keep[1]])

        def half(q):
            return 0 if (q[1] > 0 or (q[1] == 0 and q[0] > 0)) else 1

        def cmp(p, q):
            rp, rq = rel(p), rel(q)
            hp, hq = half(rp), half(rq)
            if hp != hq:
                return hp - hq
            cr = rp[0] * rq[1] - rp[1] * rq[0]
            return -1 if cr > 0 else (1 if cr < 0 else 0)

        on.sort(key=functools.cmp_to_key(cmp))
        p0 = _sub(on[0], c)
        for i in range(1, len(on) - 1):
            vol += abs(_det(p0, _sub(on[i], c), _sub(on[i + 1], c))) / 6
    return vol


def tet_box_volume(v, lo, hi) -> Fr:
    """Exact |T cap [lo,hi]| for rational vertex coordinates."""
    return polytope_volume(tet_halfspaces(v) + box_halfspaces(lo, hi))
