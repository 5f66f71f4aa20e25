"""Host-side checks of bench.py: the one-GPU contract and the frozen work model."""

import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_work_model_is_the_frozen_one():
    # 60 per tet, 24 per bbox cell, 4 per vertex-plane visit, 9 per cut,
    # 20 per sub-tetrahedron, 2 per non-zero deposit
    cnt = {"n_tet": 2, "n_pair": 10, "n_pv": 100, "n_cut": 30, "n_sub": 7, "n_nonzero": 5}
    want = (60 * 2 + 24 * 10 + 4 * 100 + 9 * 30 + 20 * 7 + 2 * 5) / 2
    assert bench.algorithmic_ops_per_tet(cnt) == want
    assert bench.PEAK_VALU_OPS == 256 * 64 * 2.4e9
