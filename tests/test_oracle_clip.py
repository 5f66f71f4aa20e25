"""Pins of the oracle's exact tetrahedron-cell intersection (Section 6.3 quantity).

Each check is fixed by mathematics independent of the oracle: closed forms,
a hand-derived worked example, exact rational vertex enumeration, partition
of unity and Monte Carlo counts.
"""

import math
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

from tests.exact_polytope import tet_box_volume

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _vol(v):
    v = np.asarray(v, float)
    return abs(np.linalg.det(np.stack([v[1] - v[0], v[2] - v[0], v[3] - v[0]]))) / 6.0


def test_worked_example_freudenthal_two_cells(orc):
    """Identity Freudenthal tet of a side-2 cube: fractions 1/8, 3/8, 3/8, 1/8 (golden file)."""
    v = np.array([[0, 0, 0], [2, 0, 0], [2, 2, 0], [2, 2, 2]], float)
    rows = [l.split() for l in open(os.path.join(GOLDEN, "freudenthal_2cell.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 8
    for x, y, z, num, den in rows:
        lo = np.array([int(x), int(y), int(z)], float)
        want = float(Fr(int(num), int(den)))
        got = orc.clip_tet_box(v, lo, lo + 1) / (4.0 / 3.0)
        assert abs(got - want) <= 1e-14, (x, y, z, got, want)
        gp = orc.clip_tet_box_paper(v, lo, lo + 1)[0] / (4.0 / 3.0)
        assert abs(gp - want) <= 1e-14, (x, y, z, gp, want)


@pytest.mark.parametrize("a", [0.0, 0.3, 0.999, 1.0, 1.25, 1.5, 2.0, 2.7, 3.0, 3.5])
def test_corner_simplex_irwin_hall(orc, a):
    """{x,y,z>=0, x+y+z<=a} cap unit cube = Irwin-Hall CDF at a (for a<=3; 1 beyond)."""
    v = np.array([[0, 0, 0], [a, 0, 0], [0, a, 0], [0, 0, a]], float)
    if a == 0.0:
        return
    want = sum((-1) ** k * math.comb(3, k) * (a - k) ** 3 for k in range(int(math.floor(min(a, 3))) + 1)) / 6.0
    if a >= 3.0:
        want = 1.0
    for fn in (orc.clip_tet_box, lambda *x: orc.clip_tet_box_paper(*x)[0]):
        got = fn(v, np.zeros(3), np.ones(3))
        assert abs(got - want) <= 1e-13 * max(1.0, want), (a, got, want)


def test_tet_inside_cell_and_cell_inside_tet(orc):
    rng = np.random.default_rng(11)
    for _ in range(50):
        v = rng.uniform(0.05, 0.95, size=(4, 3))
        assert abs(orc.clip_tet_box(v, np.zeros(3), np.ones(3)) - _vol(v)) <= 1e-15
    big = np.array([[-1, -1, -1], [6, -1, -1], [-1, 6, -1], [-1, -1, 6]], float)
    assert abs(orc.clip_tet_box(big, np.zeros(3), np.ones(3)) - 1.0) <= 1e-14
    assert abs(orc.clip_tet_box_paper(big, np.zeros(3), np.ones(3))[0] - 1.0) <= 1e-13
    far = big + 20.0
    assert orc.clip_tet_box(far, np.zeros(3), np.ones(3)) == 0.0


def _random_tets(rng, n):
    """Random, sliver, inverted-order and huge tetrahedra in cell units."""
    out = []
    for i in range(n):
        kind = i % 4
        if kind == 0:
            v = rng.uniform(-2, 4, size=(4, 3))
        elif kind == 1:  # sliver: nearly coplanar
            base = rng.uniform(-3, 5, size=(3, 3))
            w = rng.uniform(0, 1, size=3)
            w /= w.sum()
            top = w @ base + rng.normal(scale=0.02, size=3)
            v = np.vstack([base, top])
        elif kind == 2:  # swapped vertex order (negative determinant)
            v = rng.uniform(-1, 3, size=(4, 3))[[1, 0, 2, 3]]
        else:  # huge and stretched
            v = rng.uniform(-1, 2, size=(4, 3)) * np.array([9.0, 2.0, 5.0])
        out.append(v)
    return out


def test_partition_of_unity(orc):
    """Sum over the bbox cells of |T cap C| equals |T|."""
    rng = np.random.default_rng(12)
    for v in _random_tets(rng, 24):
        lo = np.floor(v.min(0)).astype(int)
        hi = np.floor(v.max(0)).astype(int)
        tot = 0.0
        totp = 0.0
        for a in range(lo[0], hi[0] + 1):
            for b in range(lo[1], hi[1] + 1):
                for c in range(lo[2], hi[2] + 1):
                    cl = np.array([a, b, c], float)
                    tot += orc.clip_tet_box(v, cl, cl + 1)
                    totp += orc.clip_tet_box_paper(v, cl, cl + 1)[0]
        V = _vol(v)
        assert abs(tot - V) <= 1e-12 * max(V, 1e-300), (tot, V)
        assert abs(totp - V) <= 1e-11 * max(V, 1e-300), (totp, V)


def test_exact_rational_vertex_enumeration(orc):
    """Dyadic inputs: the oracle matches an exact Fraction computation."""
    rng = np.random.default_rng(13)
    n_checked = 0
    for trial in range(60):
        v = rng.integers(-8, 24, size=(4, 3)) / 8.0
        if abs(np.linalg.det(np.stack([v[1] - v[0], v[2] - v[0], v[3] - v[0]]))) < 1e-3:
            continue
        cell = rng.integers(0, 2, size=3)
        lo, hi = cell.astype(float), cell.astype(float) + 1
        exact = tet_box_volume([[Fr(x).limit_denominator(64) for x in p] for p in v],
                               [Fr(int(x)) for x in lo], [Fr(int(x)) for x in hi])
        got = orc.clip_tet_box(v, lo, hi)
        gotp = orc.clip_tet_box_paper(v, lo, hi)[0]
        ref = float(exact)
        assert abs(got - ref) <= 1e-14 * max(1.0, _vol(v)), (v, cell, got, ref)
        assert abs(gotp - ref) <= 1e-13 * max(1.0, _vol(v)), (v, cell, gotp, ref)
        n_checked += 1
    assert n_checked >= 40


def test_monte_carlo_fractions(orc):
    """Uniform points in T binned per cell agree with |T cap C|/|T| within 5 sigma."""
    rng = np.random.default_rng(14)
    v = np.array([[0.3, 0.2, 0.1], [3.1, 0.7, 0.4], [1.2, 2.6, 0.9], [0.8, 1.1, 2.4]])
    n = 4_000_000
    w = rng.exponential(size=(n, 4))
    w /= w.sum(1, keepdims=True)
    pts = w @ v
    cells = np.floor(pts).astype(np.int64)
    lo = cells.min(0)
    key = ((cells[:, 0] - lo[0]) * 16 + (cells[:, 1] - lo[1])) * 16 + (cells[:, 2] - lo[2])
    counts = np.bincount(key, minlength=16 ** 3)
    V = _vol(v)
    hi = np.floor(v.max(0)).astype(int)
    for a in range(lo[0], hi[0] + 1):
        for b in range(lo[1], hi[1] + 1):
            for c in range(lo[2], hi[2] + 1):
                cl = np.array([a, b, c], float)
                p = orc.clip_tet_box(v, cl, cl + 1) / V
                k = counts[((a - lo[0]) * 16 + (b - lo[1])) * 16 + (c - lo[2])]
                sd = math.sqrt(n * p * (1 - p)) + 1.0
                assert abs(k - n * p) <= 5 * sd, (a, b, c, k, n * p)


def test_paper_scheme_counts_hand_counted(orc):
    """Visits, edge cuts and sub-tetrahedra of the paper-scheme clip (Section 6.3) equal
    the hand counts of the golden file: a tetrahedron inside the cell, the corner simplex
    at a = 3/2, and the identity Freudenthal tetrahedron of a side-2 cube in each of its
    8 cells.  These counts price the paper's algorithmic work, so a double-counted visit
    or a miscounted prism cut fails here."""
    cases = {
        "A": np.array([[0.1, 0.1, 0.1], [0.5, 0.1, 0.1], [0.1, 0.5, 0.1], [0.1, 0.1, 0.5]]),
        "B": np.array([[0, 0, 0], [1.5, 0, 0], [0, 1.5, 0], [0, 0, 1.5]], float),
        "C": np.array([[0, 0, 0], [2, 0, 0], [2, 2, 0], [2, 2, 2]], float),
    }
    rows = [l.split() for l in open(os.path.join(GOLDEN, "paper_scheme_counts.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 10
    for case, x, y, z, visits, cuts, subs in rows:
        lo = np.array([int(x), int(y), int(z)], float)
        _, pv, cut, sub = orc.clip_tet_box_paper(cases[case], lo, lo + 1)
        assert (pv, cut, sub) == (int(visits), int(cuts), int(subs)), (case, x, y, z)
