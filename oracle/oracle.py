"""ctypes binding of the C oracle (test infrastructure only).

Every function here follows the paper's definition of the result (Section 2,
Eq. (1), cell-averaged) and is documented in ``psd_oracle.h``.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "psd_oracle.c")
LIB = os.path.join(HERE, "libpsd_oracle.so")

TRIVIAL = 1
PAPER = 2

NODE_DTYPE = np.dtype([("level", "<i4"), ("ix", "<i4"), ("iy", "<i4"), ("iz", "<i4"),
                       ("first_child", "<i4"), ("leaf_id", "<i4"), ("count", "<i8")])


def build_oracle(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
               "-Wall", "-o", tmp, SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


class Counters(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "n_tet", "n_pair", "n_nontrivial", "n_nonzero", "n_inverted", "n_degenerate",
        "n_ambiguous", "n_pv", "n_cut", "n_sub")]

    def as_dict(self) -> dict:
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build_oracle(force=False)
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        lp = C.POINTER(C.c_int64)
        L.orc_clip_tet_box.restype = C.c_double
        L.orc_clip_tet_box.argtypes = [dp, dp, dp]
        L.orc_clip_tet_box_paper.restype = C.c_double
        L.orc_clip_tet_box_paper.argtypes = [dp, dp, dp, lp]
        L.orc_cube_tets.restype = None
        L.orc_cube_tets.argtypes = [C.c_void_p, ip, C.c_double, ip, C.c_int64, C.c_int64,
                                    C.c_int64, dp, dp]
        L.orc_deposit_uniform.restype = C.c_int
        L.orc_deposit_uniform.argtypes = [C.c_void_p, ip, C.c_double, C.c_double, ip, ip, ip,
                                          lp, C.c_int64, C.c_int, C.c_int, dp,
                                          C.POINTER(Counters)]
        L.orc_build_octree.restype = C.c_int
        L.orc_build_octree.argtypes = [C.c_void_p, ip, C.c_double, C.c_int, C.c_int, C.c_int,
                                       C.c_int64, C.c_void_p, C.c_int64, lp, lp]
        L.orc_deposit_octree.restype = C.c_int
        L.orc_deposit_octree.argtypes = [C.c_void_p, ip, C.c_double, C.c_double, C.c_int,
                                         C.c_void_p, C.c_int64, lp, C.c_int64, C.c_int, C.c_int,
                                         dp, C.POINTER(Counters)]
        L.orc_surrogate_examples.restype = C.c_int
        L.orc_surrogate_examples.argtypes = [C.c_void_p, ip, C.c_double, ip, C.c_int64,
                                             C.c_int64, C.c_int, C.c_void_p, C.c_void_p,
                                             C.c_void_p, dp, C.c_void_p]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(seq):
    arr = (C.c_int * len(seq))(*[int(x) for x in seq])
    return arr


def _pos(pos: np.ndarray) -> np.ndarray:
    pos = np.ascontiguousarray(pos, dtype=np.float32)
    if pos.ndim != 4 or pos.shape[3] != 3:
        raise ValueError("positions must be float32 [np0, np1, np2, 3]")
    return pos


def clip_tet_box(v, lo, hi) -> float:
    """|T cap box| by the face-list polytope clipper (Section 6.3 quantity)."""
    v = np.ascontiguousarray(v, dtype=np.float64).reshape(12)
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    return lib().orc_clip_tet_box(_dp(v), _dp(lo), _dp(hi))


def clip_tet_box_paper(v, lo, hi):
    """|T cap box| by the paper's iterative splitting; returns (V, visits, cuts, subtets)."""
    v = np.ascontiguousarray(v, dtype=np.float64).reshape(12)
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    cnt = np.zeros(3, dtype=np.int64)
    V = lib().orc_clip_tet_box_paper(_dp(v), _dp(lo), _dp(hi),
                                     cnt.ctypes.data_as(C.POINTER(C.c_int64)))
    return V, int(cnt[0]), int(cnt[1]), int(cnt[2])


def cube_tets(pos, nc, i, j, k, box: float = 1.0):
    """The 6 unwrapped tetrahedra of Lagrangian cube (i,j,k), in cell units: (tets[6,4,3], D[6])."""
    pos = _pos(pos)
    tets = np.zeros((6, 4, 3), dtype=np.float64)
    det = np.zeros(6, dtype=np.float64)
    lib().orc_cube_tets(pos.ctypes.data, _ip(pos.shape[:3]), box, _ip(nc), i, j, k,
                        _dp(tets), _dp(det))
    return tets, det


def deposit_uniform(pos, nc, box: float = 1.0, mass: float = 1.0, region=None, cubes=None,
                    mode: int = TRIVIAL, nthreads: int = 0):
    """Cell masses (float64) of the periodic grid nc (or of region=(lo, n)); returns (out, counters)."""
    pos = _pos(pos)
    nc = [int(x) for x in (nc if np.ndim(nc) else (nc, nc, nc))]
    if region is None:
        rlo, rn = None, None
        shape = tuple(nc)
    else:
        rlo, rn = _ip(region[0]), _ip(region[1])
        shape = tuple(int(x) for x in region[1])
    out = np.zeros(shape, dtype=np.float64)
    cnt = Counters()
    if cubes is not None:
        cubes = np.ascontiguousarray(cubes, dtype=np.int64)
        cptr, ncub = cubes.ctypes.data_as(C.POINTER(C.c_int64)), cubes.size
    else:
        cptr, ncub = None, 0
    rc = lib().orc_deposit_uniform(pos.ctypes.data, _ip(pos.shape[:3]), box, mass, _ip(nc),
                                   rlo, rn, cptr, ncub, mode, nthreads, _dp(out), C.byref(cnt))
    if rc != 0:
        raise ValueError(f"orc_deposit_uniform failed ({rc})")
    return out, cnt.as_dict()


def build_octree(pos, block: int = 16, max_level: int = 4, subblock: int = 8,
                 threshold: int = 1 << 20, box: float = 1.0) -> np.ndarray:
    """Canonical octree node array (structured NODE_DTYPE)."""
    pos = _pos(pos)
    nn = C.c_int64(0)
    nl = C.c_int64(0)
    rc = lib().orc_build_octree(pos.ctypes.data, _ip(pos.shape[:3]), box, block, max_level,
                                subblock, threshold, None, 0, C.byref(nn), C.byref(nl))
    if rc not in (0, -3):
        raise ValueError(f"orc_build_octree failed ({rc})")
    nodes = np.zeros(nn.value, dtype=NODE_DTYPE)
    rc = lib().orc_build_octree(pos.ctypes.data, _ip(pos.shape[:3]), box, block, max_level,
                                subblock, threshold, nodes.ctypes.data, nodes.size,
                                C.byref(nn), C.byref(nl))
    if rc != 0:
        raise ValueError(f"orc_build_octree failed ({rc})")
    return nodes


def deposit_octree(pos, nodes: np.ndarray, leaves, block: int = 16, box: float = 1.0,
                   mass: float = 1.0, mode: int = TRIVIAL, nthreads: int = 0):
    """Cell masses of the selected leaves: float64 [len(leaves), B, B, B]; returns (out, counters)."""
    pos = _pos(pos)
    nodes = np.ascontiguousarray(nodes, dtype=NODE_DTYPE)
    leaves = np.ascontiguousarray(leaves, dtype=np.int64)
    out = np.zeros((leaves.size, block, block, block), dtype=np.float64)
    cnt = Counters()
    rc = lib().orc_deposit_octree(pos.ctypes.data, _ip(pos.shape[:3]), box, mass, block,
                                  nodes.ctypes.data, nodes.size,
                                  leaves.ctypes.data_as(C.POINTER(C.c_int64)), leaves.size,
                                  mode, nthreads, _dp(out), C.byref(cnt))
    if rc != 0:
        raise ValueError(f"orc_deposit_octree failed ({rc})")
    return out, cnt.as_dict()


def surrogate_examples(pos, nc, box: float = 1.0, first: int = 0, count: int | None = None,
                       nthreads: int = 0, compact: bool = True) -> dict:
    """Eligible tetrahedra (bbox within 2 cells per axis) of cubes first..first+count-1 with
    their features float(v - lo), cell masks, exact overlap fractions |T cap C|/|T| and
    bbox origins lo (wrapped into [0, nc)).

    compact=True keeps only the eligible ones, in canonical order (cube, then split
    permutation); "tet" holds their global tetrahedron index 6*cube + p."""
    pos = _pos(pos)
    nc = [int(x) for x in (nc if np.ndim(nc) else (nc, nc, nc))]
    ncube = int(np.prod(pos.shape[:3]))
    if count is None:
        count = ncube - first
    n = 6 * count
    flag = np.zeros(n, dtype=np.uint8)
    feat = np.zeros((n, 12), dtype=np.float32)
    mask = np.zeros(n, dtype=np.uint8)
    frac = np.zeros((n, 8), dtype=np.float64)
    lo = np.zeros((n, 3), dtype=np.int32)
    rc = lib().orc_surrogate_examples(pos.ctypes.data, _ip(pos.shape[:3]), box, _ip(nc), first,
                                      count, nthreads, flag.ctypes.data, feat.ctypes.data,
                                      mask.ctypes.data, _dp(frac), lo.ctypes.data)
    if rc != 0:
        raise ValueError("orc_surrogate_examples: bad arguments")
    tet = np.arange(6 * first, 6 * (first + count), dtype=np.int64)
    out = {"flag": flag, "feat": feat, "mask": mask, "frac": frac, "lo": lo, "tet": tet}
    if compact:
        keep = flag.astype(bool)
        out = {k: v[keep] for k, v in out.items() if k != "flag"}
    return out
