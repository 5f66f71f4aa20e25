"""Host-side checks of bench.py: the one-GPU contract and the frozen work models."""

import os
import subprocess
import sys

import bench
import costmodel

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_paper_work_model_is_the_frozen_one():
    # 60 per tet, 24 per bbox cell, 4 per vertex-plane visit, 9 per cut,
    # 20 per sub-tetrahedron, 2 per non-zero deposit
    cnt = {"n_tet": 2, "n_pair": 10, "n_pv": 100, "n_cut": 30, "n_sub": 7, "n_nonzero": 5}
    want = (60 * 2 + 24 * 10 + 4 * 100 + 9 * 30 + 20 * 7 + 2 * 5) / 2
    assert bench.paper_ops_per_tet(cnt) == want
    assert bench.PEAK_VALU_OPS == 256 * 64 * 2.4e9


def test_own_work_model_is_the_frozen_one():
    # unit costs of the cumulative kernel's events, fixed before any measurement
    assert costmodel.COST == {"tet": 250, "column": 137, "xpiece": 110, "piece": 122,
                              "level": 6, "colcell": 15, "nz": 5}
    ev = {"tet": 1, "column": 2, "xpiece": 3, "piece": 4, "level": 5, "colcell": 6, "nz": 7}
    assert costmodel.own_ops(ev) == 250 + 2 * 137 + 3 * 110 + 4 * 122 + 5 * 6 + 6 * 15 + 7 * 5


def test_roofline_terms_and_fraction():
    own = {"ops_per_tet": 1000.0}
    peaks = {"global_atomic_add_f32_tile_rows": 1e10, "global_atomic_add_f32_random": 5e9,
             "global_atomic_add_f32_coalesced": 4e10}
    # 1e6 tets in 10 ms: 1e9 ops -> 1e11 op/s against 3.93e13
    r = bench.roofline_line("k", 10.0, 10 ** 6, own, 2000.0, 5e7, 8e9, peaks, None, None)
    assert abs(r["frac"] - 1e11 / bench.PEAK_VALU_OPS) < 1e-15
    assert r["bound"] == "alu"
    # terms: valu 1e9 / 3.93e13 = 25 us, atomics 5e7 / 1e10 = 5 ms, HBM 8e9 / 8e12 = 1 ms
    assert r["binding_term"] == "atomic"
    assert abs(r["frac_of_max_term"] - 0.5) < 1e-12
    assert abs(r["atomic"]["frac"] - 0.5) < 1e-12
    assert abs(r["paper_method_equivalent"]["ops_per_tet"] - 2000.0) < 1e-12
