"""Pins of the oracle's depositor (Section 2 Eq. (1) cell-averaged; Section 6.1 loop).

Invariants fixed by the definition M_C = sum_T m |T cap C| / |T|: mass
conservation, uniform density of an undisplaced lattice, a tetrahedron inside
one cell, periodic shifts, relabelling, the orientation-sum identity of the
tessellation, and agreement of the short-cut and plain loops.
"""

import numpy as np
import pytest

from synth import (jittered_lattice_positions, lattice_positions, zeldovich_positions)


def _quantize(pos, bits=16):
    """Snap positions to multiples of 2^-bits so dyadic shifts stay exact in float32."""
    q = np.round(pos.astype(np.float64) * (1 << bits)) / (1 << bits)
    q = np.mod(q, 1.0).astype(np.float32)
    return q


@pytest.mark.parametrize("nc", [64, 16, 24])
def test_undisplaced_lattice_gives_uniform_density(orc, nc):
    pos = lattice_positions(32)
    out, cnt = orc.deposit_uniform(pos, nc, mass=1.0)
    rho = out * nc ** 3
    assert np.max(np.abs(rho - 1.0)) <= 1e-12
    assert cnt["n_tet"] == 6 * 32 ** 3
    assert cnt["n_inverted"] == 0 and cnt["n_degenerate"] == 0


def test_mass_conservation_and_orientation_sum(orc):
    pos = zeldovich_positions(16, 0.5, seed=21)
    nc = 32
    out, cnt = orc.deposit_uniform(pos, nc, mass=2.5)
    assert abs(out.sum() - 2.5) <= 1e-12 * 2.5
    # Sum over the tessellation of the volumes signed relative to the undeformed
    # lattice's orientation = box volume (cells^3): the periodic map has degree 1.
    ref_sign = np.array([1, -1, -1, 1, 1, -1], float)  # parities of 012,021,102,120,201,210
    tot = 0.0
    for i in range(16):
        for j in range(16):
            for k in range(16):
                _, D = orc.cube_tets(pos, (nc, nc, nc), i, j, k)
                tot += (ref_sign * D).sum() / 6.0
    assert abs(tot - nc ** 3) <= 1e-9 * nc ** 3


def test_shortcut_and_plain_loops_agree(orc):
    pos = zeldovich_positions(8, 0.8, seed=22)
    a, ca = orc.deposit_uniform(pos, 16, mode=orc.TRIVIAL)
    b, cb = orc.deposit_uniform(pos, 16, mode=0)
    c, cc = orc.deposit_uniform(pos, 16, mode=orc.TRIVIAL | orc.PAPER)
    assert np.max(np.abs(a - b)) <= 1e-15
    assert np.max(np.abs(a - c)) <= 1e-13
    assert ca["n_pair"] == cb["n_pair"] == cc["n_pair"]
    assert cc["n_pv"] > 0 and cc["n_sub"] > 0


def test_tet_inside_one_cell_puts_all_mass_there(orc):
    # A lattice so fine that every cube sits inside one cell of a coarse grid.
    np_ = 8
    pos = lattice_positions(np_).astype(np.float64)
    pos = (pos * 0.5 + 0.1).astype(np.float32)   # compress into [0.1, 0.5)
    # grid of 2 cells: all particles except the periodic wrap layer are in cell 0
    out, _ = orc.deposit_uniform(pos[:, :, :, :], 2, mass=1.0,
                                 cubes=np.array([0, 1, 8, 9], dtype=np.int64))
    m = 1.0 / (6 * np_ ** 3)
    assert abs(out[0, 0, 0] - 4 * 6 * m) <= 1e-17
    assert np.count_nonzero(out) == 1


def test_integer_cell_shift_rolls_output(orc):
    pos = _quantize(zeldovich_positions(12, 0.7, seed=23))
    nc = 32
    base, _ = orc.deposit_uniform(pos, nc)
    shift = np.array([3, -5, 7])
    sh = np.mod(pos.astype(np.float64) + shift / nc, 1.0).astype(np.float32)
    assert np.array_equal(np.mod(sh.astype(np.float64) - shift / nc, 1.0).astype(np.float32), pos)
    moved, _ = orc.deposit_uniform(sh, nc)
    assert np.max(np.abs(np.roll(base, tuple(shift), axis=(0, 1, 2)) - moved)) <= 1e-13


def test_periodic_image_of_particles_is_irrelevant(orc):
    pos = _quantize(zeldovich_positions(12, 0.7, seed=24))
    base, _ = orc.deposit_uniform(pos, 24)
    rng = np.random.default_rng(5)
    alt = pos.copy()
    sel = rng.random(pos.shape[:3]) < 0.3
    alt[sel] += np.float32(1.0)
    sel2 = rng.random(pos.shape[:3]) < 0.2
    alt[sel2] -= np.float32(1.0)
    moved, _ = orc.deposit_uniform(alt, 24)
    assert np.max(np.abs(base - moved)) <= 1e-13


def test_relabelling_lagrangian_grid_is_irrelevant(orc):
    pos = zeldovich_positions(12, 0.9, seed=25)
    base, _ = orc.deposit_uniform(pos, 20)
    rolled = np.ascontiguousarray(np.roll(pos, (4, -3, 5), axis=(0, 1, 2)))
    moved, _ = orc.deposit_uniform(rolled, 20)
    assert np.max(np.abs(base - moved)) <= 1e-13


def test_jittered_lattice_conserves_mass(orc):
    """Analytic input of the paper's weak-scaling runs (offsets up to one cell)."""
    pos = jittered_lattice_positions(16, 1.0, seed=26)
    out, cnt = orc.deposit_uniform(pos, 16)
    assert abs(out.sum() - 1.0) <= 1e-12
    zero = jittered_lattice_positions(16, 0.0, seed=26)
    out0, _ = orc.deposit_uniform(zero, 16)
    assert np.max(np.abs(out0 * 16 ** 3 - 1.0)) <= 1e-12


def test_region_matches_full_grid(orc):
    pos = zeldovich_positions(12, 1.0, seed=27)
    full, _ = orc.deposit_uniform(pos, 24)
    part, _ = orc.deposit_uniform(pos, 24, region=((5, 0, 17), (7, 24, 7)))
    assert np.max(np.abs(full[5:12, :, 17:24] - part)) <= 1e-15


def test_cube_subset_sums_to_whole(orc):
    pos = zeldovich_positions(8, 0.6, seed=28)
    full, _ = orc.deposit_uniform(pos, 16)
    ids = np.arange(8 ** 3)
    a, _ = orc.deposit_uniform(pos, 16, cubes=ids[::2])
    b, _ = orc.deposit_uniform(pos, 16, cubes=ids[1::2])
    assert np.max(np.abs(full - (a + b))) <= 1e-15


def test_degenerate_tets_go_to_centroid_cell(orc):
    # All particles of a plane collapsed: tets of the cubes touching it are flat.
    pos = lattice_positions(8).astype(np.float64)
    pos[:, :, :, 2] = 0.3          # every particle at z = 0.3 -> all tets flat
    pos = pos.astype(np.float32)
    out, cnt = orc.deposit_uniform(pos, 8)
    assert cnt["n_degenerate"] == cnt["n_tet"]
    assert abs(out.sum() - 1.0) <= 1e-12
    assert np.all(out[:, :, 2] > 0) and np.count_nonzero(out.sum(axis=(0, 1))) == 1
