"""Phase-space-element density deposition on AMD MI355X (gfx950).

Thin ctypes binding of ``libpsd.so`` (C ABI in ``include/psd.h``).  Every
step of the deposition runs in the library's HIP kernels; this module only
allocates outputs and workspaces with PyTorch and passes pointers and the
current HIP stream.  There is no CPU fallback: if the library is missing the
calls raise.
"""

from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpsd.so")

PSD_OK = 0
PSD_ERR_ARG = -1
PSD_ERR_WORKSPACE = -2
PSD_ERR_CAPACITY = -3
PSD_ERR_NONFINITE = -4
PSD_ERR_UNSUPPORTED = -5
PSD_ERR_HIP = -6

PSD_OUT_DENSITY = 1 << 0
PSD_ACCUMULATE = 1 << 1
PSD_PREC_FP64 = 1 << 2
PSD_METHOD_CELL = 1 << 3
PSD_SURROGATE = 1 << 4
PSD_CHECK_FINITE = 1 << 5
PSD_WORK_COUNTERS = 1 << 6
PSD_METHOD_SLAB = 1 << 7

PSD_SURROGATE_PARAMS = 9672

STAT_NAMES = ("tets", "pairs", "clips_or_columns", "nonzero", "inverted", "degenerate",
              "surrogate_tets", "dropped_nonfinite")
# stats[8..11] with PSD_WORK_COUNTERS (the stats tensor then has 16 entries)
WORK_STAT_NAMES = ("xpieces", "pieces", "levels", "column_levels")


class PsdError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__(f"{where}: {code} ({detail})")
        self.code = code


class Particles(C.Structure):
    _fields_ = [("np", C.c_int32 * 3), ("box", C.c_double), ("total_mass", C.c_double)]


class Tuning(C.Structure):
    _fields_ = [("lds_cap", C.c_int32), ("waves_per_cu", C.c_int32), ("ordered", C.c_int32),
                ("reserved", C.c_int32)]


class Options(C.Structure):
    _fields_ = [("flags", C.c_uint32), ("stats", C.c_void_p), ("tuning", C.POINTER(Tuning)),
                ("surrogate", C.c_void_p)]


def _options(flags: int, stats, tuning, surrogate=None) -> Options:
    o = Options(flags, stats.data_ptr() if stats is not None else None, None,
                surrogate.data_ptr() if surrogate is not None else None)
    if tuning is not None:
        t = Tuning(*[int(x) for x in tuning], 0) if not isinstance(tuning, Tuning) else tuning
        o._tuning_ref = t
        o.tuning = C.pointer(t)
    return o


_lib = None


def lib() -> C.CDLL:
    """The loaded libpsd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "or python -m paper_1612_09491_amd.build")
        L = C.CDLL(LIB_PATH)
        L.psd_status_string.restype = C.c_char_p
        L.psd_status_string.argtypes = [C.c_int]
        L.psd_last_error_detail.restype = C.c_char_p
        L.psd_last_error_detail.argtypes = []
        L.psd_uniform_workspace_size.restype = C.c_int
        L.psd_uniform_workspace_size.argtypes = [C.POINTER(Particles), C.POINTER(C.c_int32),
                                                 C.POINTER(Options), C.POINTER(C.c_size_t)]
        L.psd_deposit_uniform.restype = C.c_int
        L.psd_deposit_uniform.argtypes = [C.c_void_p, C.POINTER(Particles),
                                          C.POINTER(C.c_int32), C.c_void_p, C.c_void_p,
                                          C.POINTER(Options), C.c_void_p, C.c_size_t,
                                          C.c_void_p]
        _lib = L
    return _lib


def _check(code: int, where: str) -> None:
    if code != PSD_OK:
        detail = lib().psd_last_error_detail().decode(errors="replace")
        raise PsdError(code, where, detail)


def _grid3(nc) -> tuple[int, int, int]:
    if isinstance(nc, int):
        return (nc, nc, nc)
    t = tuple(int(x) for x in nc)
    if len(t) != 3:
        raise ValueError("grid size must be an int or 3 ints")
    return t


def _check_aux(mass_sum, n_sums: int, stats, flags: int = 0) -> None:
    """The optional device outputs every deposit takes: FP64 mass sums (n_sums of them)
    and the int64 counters (8 of them, 16 with PSD_WORK_COUNTERS); the kernels add into
    them with 8-byte atomics."""
    if mass_sum is not None and (not isinstance(mass_sum, torch.Tensor) or
                                 mass_sum.dtype != torch.float64 or not mass_sum.is_cuda or
                                 not mass_sum.is_contiguous() or mass_sum.numel() < n_sums):
        raise ValueError(f"mass_sum must be a contiguous CUDA float64 tensor with {n_sums} "
                         f"entr{'y' if n_sums == 1 else 'ies'}")
    n_stats = 16 if flags & PSD_WORK_COUNTERS else 8
    if stats is not None and (not isinstance(stats, torch.Tensor) or stats.dtype != torch.int64 or
                              not stats.is_cuda or not stats.is_contiguous() or
                              stats.numel() < n_stats):
        raise ValueError(f"stats must be a contiguous CUDA int64 tensor with {n_stats} entries")


def _workspace(workspace, nbytes: int, device) -> torch.Tensor:
    """The caller's workspace (a CUDA tensor of at least nbytes bytes) or a new one."""
    if workspace is None:
        return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
    if not isinstance(workspace, torch.Tensor) or not workspace.is_cuda or \
            not workspace.is_contiguous() or workspace.numel() * workspace.element_size() < nbytes:
        raise ValueError(f"workspace must be a contiguous CUDA tensor of at least {nbytes} bytes")
    return workspace


def _stream_handle(stream) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def _particles(pos: torch.Tensor, box: float, mass: float) -> Particles:
    if not pos.is_cuda or pos.dtype != torch.float32 or pos.dim() != 4 or pos.shape[3] != 3:
        raise ValueError("pos must be a CUDA float32 tensor [np0, np1, np2, 3]")
    if not pos.is_contiguous():
        raise ValueError("pos must be contiguous")
    p = Particles()
    for a in range(3):
        p.np[a] = int(pos.shape[a])
    p.box = float(box)
    p.total_mass = float(mass)
    return p


def uniform_workspace_size(np_, nc, flags: int = 0, box: float = 1.0, mass: float = 1.0,
                           tuning=None) -> int:
    p = Particles()
    for a, n in enumerate(_grid3(np_)):
        p.np[a] = n
    p.box, p.total_mass = float(box), float(mass)
    ncs = (C.c_int32 * 3)(*_grid3(nc))
    o = _options(flags, None, tuning)
    nbytes = C.c_size_t(0)
    _check(lib().psd_uniform_workspace_size(C.byref(p), ncs, C.byref(o), C.byref(nbytes)),
           "psd_uniform_workspace_size")
    return int(nbytes.value)


def deposit_uniform(pos: torch.Tensor, nc, box: float = 1.0, mass: float = 1.0, flags: int = 0,
                    out: torch.Tensor | None = None, mass_sum: torch.Tensor | None = None,
                    stats: torch.Tensor | None = None, workspace: torch.Tensor | None = None,
                    stream=None, tuning=None, surrogate: torch.Tensor | None = None) -> torch.Tensor:
    """Cell masses (or densities with PSD_OUT_DENSITY) on a periodic nc grid.

    Returns ``out`` (float32, or float64 with PSD_PREC_FP64).  ``mass_sum``
    (float64[1]) receives the FP64 sum of deposited mass; ``stats`` (int64[8])
    receives counters (see STAT_NAMES).  With PSD_SURROGATE, ``surrogate`` is
    the network's packed float32 parameters.  Asynchronous on the current stream.
    """
    if surrogate is not None:
        _check_params(surrogate)
    p = _particles(pos, box, mass)
    g = _grid3(nc)
    dtype = torch.float64 if flags & PSD_PREC_FP64 else torch.float32
    if out is None:
        out = torch.empty(g, dtype=dtype, device=pos.device)
    elif out.dtype != dtype or tuple(out.shape) != g or not out.is_contiguous() or not out.is_cuda:
        raise ValueError(f"out must be a contiguous CUDA {dtype} tensor of shape {g}")
    nbytes = uniform_workspace_size(tuple(pos.shape[:3]), g, flags, box, mass, tuning)
    workspace = _workspace(workspace, nbytes, pos.device)
    _check_aux(mass_sum, 1, stats, flags)
    o = _options(flags, stats, tuning, surrogate)
    ncs = (C.c_int32 * 3)(*g)
    _check(lib().psd_deposit_uniform(pos.data_ptr(), C.byref(p), ncs, out.data_ptr(),
                                     mass_sum.data_ptr() if mass_sum is not None else None,
                                     C.byref(o), workspace.data_ptr(),
                                     workspace.numel() * workspace.element_size(),
                                     _stream_handle(stream)),
           "psd_deposit_uniform")
    return out


PSD_NOALLOC_SCRATCH_BYTES = 16 << 20


def deposit_uniform_noalloc(pos: torch.Tensor, nc, box: float = 1.0, mass: float = 1.0,
                            flags: int = 0, out: torch.Tensor | None = None,
                            mass_sum: torch.Tensor | None = None,
                            stats: torch.Tensor | None = None, stream=None, tuning=None,
                            surrogate: torch.Tensor | None = None) -> torch.Tensor:
    """``deposit_uniform`` through psd_deposit_uniform_noalloc: the library's fixed
    per-GPU scratch array serves as the workspace, so the call allocates nothing
    on the device when ``out`` is given.  Calls that overlap in time on one GPU
    race on that array.  Problems needing more than PSD_NOALLOC_SCRATCH_BYTES of
    workspace raise PsdError (PSD_ERR_WORKSPACE)."""
    L = lib()
    if not getattr(L, "_noalloc_bound", False):
        L.psd_deposit_uniform_noalloc.restype = C.c_int
        L.psd_deposit_uniform_noalloc.argtypes = [C.c_void_p, C.POINTER(Particles),
                                                  C.POINTER(C.c_int32), C.c_void_p, C.c_void_p,
                                                  C.POINTER(Options), C.c_void_p]
        L._noalloc_bound = True
    if surrogate is not None:
        _check_params(surrogate)
    p = _particles(pos, box, mass)
    g = _grid3(nc)
    dtype = torch.float64 if flags & PSD_PREC_FP64 else torch.float32
    if out is None:
        out = torch.empty(g, dtype=dtype, device=pos.device)
    elif out.dtype != dtype or tuple(out.shape) != g or not out.is_contiguous() or not out.is_cuda:
        raise ValueError(f"out must be a contiguous CUDA {dtype} tensor of shape {g}")
    _check_aux(mass_sum, 1, stats, flags)
    o = _options(flags, stats, tuning, surrogate)
    ncs = (C.c_int32 * 3)(*g)
    _check(L.psd_deposit_uniform_noalloc(pos.data_ptr(), C.byref(p), ncs, out.data_ptr(),
                                         mass_sum.data_ptr() if mass_sum is not None else None,
                                         C.byref(o), _stream_handle(stream)),
           "psd_deposit_uniform_noalloc")
    return out


# ---------------------------------------------------------------------------
# Octree
# ---------------------------------------------------------------------------

class OctreeParams(C.Structure):
    _fields_ = [("block_cells", C.c_int32), ("max_level", C.c_int32), ("subblock", C.c_int32),
                ("reserved", C.c_int32), ("threshold", C.c_int64)]


NODE_BYTES = 32
NODE_FIELDS = (("level", "<i4"), ("ix", "<i4"), ("iy", "<i4"), ("iz", "<i4"),
               ("first_child", "<i4"), ("leaf_id", "<i4"), ("count", "<i8"))


def _octree_params(block, max_level, subblock, threshold) -> OctreeParams:
    return OctreeParams(int(block), int(max_level), int(subblock), 0, int(threshold))


def _bind_octree(L):
    if getattr(L, "_octree_bound", False):
        return
    L.psd_octree_workspace_size.restype = C.c_int
    L.psd_octree_workspace_size.argtypes = [C.POINTER(Particles), C.POINTER(OctreeParams),
                                            C.POINTER(C.c_size_t)]
    L.psd_build_octree.restype = C.c_int
    L.psd_build_octree.argtypes = [C.c_void_p, C.POINTER(Particles), C.POINTER(OctreeParams),
                                   C.c_void_p, C.c_int64, C.POINTER(C.c_int64),
                                   C.POINTER(C.c_int64), C.c_void_p, C.c_size_t, C.c_void_p]
    L.psd_deposit_octree.restype = C.c_int
    L.psd_deposit_octree.argtypes = [C.c_void_p, C.POINTER(Particles), C.POINTER(OctreeParams),
                                     C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p,
                                     C.POINTER(Options), C.c_void_p, C.c_size_t, C.c_void_p]
    L._octree_bound = True


def max_nodes(max_level: int) -> int:
    return sum(8 ** l for l in range(max_level + 1))


def octree_workspace_size(np_, block=16, max_level=4, subblock=8, threshold=1 << 20,
                          box: float = 1.0, mass: float = 1.0) -> int:
    L = lib()
    _bind_octree(L)
    p = Particles()
    for a, n in enumerate(_grid3(np_)):
        p.np[a] = n
    p.box, p.total_mass = float(box), float(mass)
    op = _octree_params(block, max_level, subblock, threshold)
    nbytes = C.c_size_t(0)
    _check(L.psd_octree_workspace_size(C.byref(p), C.byref(op), C.byref(nbytes)),
           "psd_octree_workspace_size")
    return int(nbytes.value)


class Octree:
    """Device node array plus its sizes and build parameters."""

    def __init__(self, nodes: torch.Tensor, n_nodes: int, n_leaves: int, block: int,
                 max_level: int, subblock: int, threshold: int):
        self.nodes, self.n_nodes, self.n_leaves = nodes, n_nodes, n_leaves
        self.block, self.max_level, self.subblock, self.threshold = block, max_level, subblock, threshold

    def to_numpy(self):
        import numpy as np
        raw = self.nodes[: self.n_nodes * NODE_BYTES].cpu().numpy()
        return raw.view(np.dtype(list(NODE_FIELDS)))


def build_octree(pos: torch.Tensor, block: int = 16, max_level: int = 4, subblock: int = 8,
                 threshold: int = 1 << 20, box: float = 1.0, capacity: int | None = None,
                 workspace: torch.Tensor | None = None, stream=None) -> Octree:
    """Adaptive octree of psd_build_octree (synchronizes the stream)."""
    L = lib()
    _bind_octree(L)
    p = _particles(pos, box, 1.0)
    op = _octree_params(block, max_level, subblock, threshold)
    cap = max_nodes(max_level) if capacity is None else int(capacity)
    nodes = torch.empty(max(cap, 1) * NODE_BYTES, dtype=torch.uint8, device=pos.device)
    nbytes = octree_workspace_size(tuple(pos.shape[:3]), block, max_level, subblock, threshold, box)
    workspace = _workspace(workspace, nbytes, pos.device)
    nn, nl = C.c_int64(0), C.c_int64(0)
    code = L.psd_build_octree(pos.data_ptr(), C.byref(p), C.byref(op), nodes.data_ptr(), cap,
                              C.byref(nn), C.byref(nl), workspace.data_ptr(),
                              workspace.numel() * workspace.element_size(),
                              _stream_handle(stream))
    if code == PSD_ERR_CAPACITY:
        err = PsdError(code, "psd_build_octree", f"needs {nn.value} nodes")
        err.n_nodes, err.n_leaves = int(nn.value), int(nl.value)
        raise err
    _check(code, "psd_build_octree")
    return Octree(nodes, int(nn.value), int(nl.value), block, max_level, subblock, threshold)


def deposit_octree(pos: torch.Tensor, tree: Octree, box: float = 1.0, mass: float = 1.0,
                   flags: int = 0, out: torch.Tensor | None = None,
                   mass_sum: torch.Tensor | None = None, stats: torch.Tensor | None = None,
                   workspace: torch.Tensor | None = None, stream=None, tuning=None) -> torch.Tensor:
    """Leaf cell masses (or densities) [n_leaves, B, B, B] float32."""
    L = lib()
    _bind_octree(L)
    p = _particles(pos, box, mass)
    op = _octree_params(tree.block, tree.max_level, tree.subblock, tree.threshold)
    B = tree.block
    shape = (tree.n_leaves, B, B, B)
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=pos.device)
    elif (out.dtype != torch.float32 or tuple(out.shape) != shape or not out.is_contiguous() or
          not out.is_cuda):
        raise ValueError(f"out must be a contiguous CUDA float32 tensor of shape {shape}")
    if not tree.nodes.is_cuda:
        raise ValueError("the octree's node array must be on the GPU")
    nbytes = octree_workspace_size(tuple(pos.shape[:3]), tree.block, tree.max_level, tree.subblock,
                                   tree.threshold, box)
    workspace = _workspace(workspace, nbytes, pos.device)
    _check_aux(mass_sum, 1, stats, flags)
    o = _options(flags, stats, tuning)
    _check(L.psd_deposit_octree(pos.data_ptr(), C.byref(p), C.byref(op), tree.nodes.data_ptr(),
                                tree.n_nodes, tree.n_leaves, out.data_ptr(),
                                mass_sum.data_ptr() if mass_sum is not None else None,
                                C.byref(o), workspace.data_ptr(),
                                workspace.numel() * workspace.element_size(),
                                _stream_handle(stream)),
           "psd_deposit_octree")
    return out


# ---------------------------------------------------------------------------
# Batched boxes and autotuning
# ---------------------------------------------------------------------------

class Box(C.Structure):
    _fields_ = [("pos", C.c_void_p), ("p", Particles), ("nc", C.c_int32 * 3), ("out", C.c_void_p)]


def _bind_batched(L):
    if getattr(L, "_batched_bound", False):
        return
    L.psd_batched_workspace_size.restype = C.c_int
    L.psd_batched_workspace_size.argtypes = [C.POINTER(Box), C.c_int32, C.POINTER(Options),
                                             C.POINTER(C.c_size_t)]
    L.psd_deposit_batched.restype = C.c_int
    L.psd_deposit_batched.argtypes = [C.POINTER(Box), C.c_int32, C.c_void_p, C.POINTER(Options),
                                      C.c_void_p, C.c_size_t, C.c_void_p]
    L.psd_autotune_batched.restype = C.c_int
    L.psd_autotune_batched.argtypes = [C.POINTER(Box), C.c_int32, C.POINTER(Options), C.c_void_p,
                                       C.c_size_t, C.c_void_p, C.c_char_p, C.POINTER(Tuning),
                                       C.POINTER(C.c_double)]
    L._batched_bound = True


def _box_array(boxes, box: float, mass: float, flags: int):
    """boxes: list of (pos tensor, nc, out tensor or None) -> (ctypes array, outs)."""
    arr = (Box * len(boxes))()
    outs = []
    for i, item in enumerate(boxes):
        pos, nc = item[0], _grid3(item[1])
        out = item[2] if len(item) > 2 else None
        p = _particles(pos, box, mass)
        if out is None:
            out = torch.empty(nc, dtype=torch.float32, device=pos.device)
        elif (out.dtype != torch.float32 or tuple(out.shape) != nc or not out.is_contiguous() or
              not out.is_cuda):
            raise ValueError(f"box {i}: out must be a contiguous CUDA float32 tensor of shape {nc}")
        arr[i].pos = pos.data_ptr()
        arr[i].p = p
        for a in range(3):
            arr[i].nc[a] = nc[a]
        arr[i].out = out.data_ptr()
        outs.append(out)
    return arr, outs


def batched_workspace_size(boxes, flags: int = 0, tuning=None, box: float = 1.0) -> int:
    L = lib()
    _bind_batched(L)
    arr, _ = _box_array(boxes, box, 1.0, flags)
    o = _options(flags, None, tuning)
    nbytes = C.c_size_t(0)
    _check(L.psd_batched_workspace_size(arr, len(arr), C.byref(o), C.byref(nbytes)),
           "psd_batched_workspace_size")
    return int(nbytes.value)


def deposit_batched(boxes, box: float = 1.0, mass: float = 1.0, flags: int = 0,
                    mass_sums: torch.Tensor | None = None, stats: torch.Tensor | None = None,
                    tuning=None, workspace: torch.Tensor | None = None, stream=None):
    """Deposit a list of independent boxes [(pos, nc[, out]), ...] in one launch.

    Every box uses the same box side and total mass.  Returns the list of
    output grids (float32).
    """
    L = lib()
    _bind_batched(L)
    arr, outs = _box_array(boxes, box, mass, flags)
    o = _options(flags, stats, tuning)
    nbytes = C.c_size_t(0)
    _check(L.psd_batched_workspace_size(arr, len(arr), C.byref(o), C.byref(nbytes)),
           "psd_batched_workspace_size")
    dev = outs[0].device
    workspace = _workspace(workspace, int(nbytes.value), dev)
    _check_aux(mass_sums, len(arr), stats, flags)
    _check(L.psd_deposit_batched(arr, len(arr), mass_sums.data_ptr() if mass_sums is not None else None,
                                 C.byref(o), workspace.data_ptr(),
                                 workspace.numel() * workspace.element_size(),
                                 _stream_handle(stream)),
           "psd_deposit_batched")
    return outs


def autotune_batched(boxes, box: float = 1.0, mass: float = 1.0, flags: int = 0,
                     cache_path: str | None = None, stream=None):
    """Best launch shape for this batch (timed on the GPU; cached when cache_path is set).

    Returns ((lds_cap, waves_per_cu, ordered), milliseconds).
    """
    L = lib()
    _bind_batched(L)
    arr, outs = _box_array(boxes, box, mass, flags)
    o = _options(flags, None, (0, 0, 1))
    nbytes = C.c_size_t(0)
    _check(L.psd_batched_workspace_size(arr, len(arr), C.byref(o), C.byref(nbytes)),
           "psd_batched_workspace_size")
    ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=outs[0].device)
    o2 = _options(flags, None, None)
    best = Tuning()
    ms = C.c_double(0.0)
    _check(L.psd_autotune_batched(arr, len(arr), C.byref(o2), ws.data_ptr(), ws.numel(),
                                  _stream_handle(stream),
                                  cache_path.encode() if cache_path else None, C.byref(best),
                                  C.byref(ms)),
           "psd_autotune_batched")
    return (best.lds_cap, best.waves_per_cu, best.ordered), float(ms.value)


# ---------------------------------------------------------------------------
# Learned overlap surrogate
# ---------------------------------------------------------------------------

SURROGATE_LAYOUT = (("W1", (64, 12)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)),
                    ("W3", (64, 64)), ("b3", (64,)), ("W4", (8, 64)), ("b4", (8,)))


def _bind_surrogate(L):
    if getattr(L, "_surrogate_bound", False):
        return
    L.psd_surrogate_examples_workspace_size.restype = C.c_int
    L.psd_surrogate_examples_workspace_size.argtypes = [C.c_int64, C.POINTER(C.c_size_t)]
    L.psd_surrogate_examples.restype = C.c_int
    L.psd_surrogate_examples.argtypes = [C.c_void_p, C.POINTER(Particles), C.POINTER(C.c_int32),
                                         C.c_int64, C.c_int64, C.c_int32, C.c_void_p, C.c_void_p,
                                         C.c_void_p, C.c_void_p, C.c_int64,
                                         C.POINTER(C.c_int64), C.c_void_p, C.c_size_t,
                                         C.c_void_p]
    L.psd_exact_fractions.restype = C.c_int
    L.psd_exact_fractions.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
    L.psd_surrogate_forward.restype = C.c_int
    L.psd_surrogate_forward.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                        C.c_void_p, C.c_void_p]
    L.psd_surrogate_backward.restype = C.c_int
    L.psd_surrogate_backward.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                         C.c_void_p]
    L.psd_surrogate_adam.restype = C.c_int
    L.psd_surrogate_adam.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                     C.c_float, C.c_float, C.c_float, C.c_float, C.c_void_p]
    L.psd_surrogate_train_steps.restype = C.c_int
    L.psd_surrogate_train_steps.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                            C.c_void_p, C.c_int64, C.c_int64, C.c_int64, C.c_int64,
                                            C.c_void_p, C.c_float, C.c_float, C.c_float, C.c_void_p,
                                            C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    L._surrogate_bound = True


def _check_params(w: torch.Tensor) -> None:
    if (not w.is_cuda or w.dtype != torch.float32 or w.numel() != PSD_SURROGATE_PARAMS or
            not w.is_contiguous()):
        raise ValueError(f"surrogate parameters must be a contiguous CUDA float32 tensor of "
                         f"{PSD_SURROGATE_PARAMS} values")


def _cuda(t: torch.Tensor, dtype, shape_tail, name: str) -> None:
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous() or tuple(t.shape[1:]) != shape_tail:
        raise ValueError(f"{name} must be a contiguous CUDA {dtype} tensor [n, *{shape_tail}]")


def surrogate_examples(pos: torch.Tensor, nc, box: float = 1.0, first_cube: int = 0,
                       n_cubes: int | None = None, min_cells: int = 2,
                       capacity: int | None = None, with_ids: bool = True, stream=None) -> dict:
    """Eligible tetrahedra (bbox within 2 cells per axis, >= min_cells cells) of the cube
    range with features [n,12], exact overlap fractions [n,8] (float64), cell masks [n]
    and tetrahedron ids [n], in tetrahedron order.  Synchronizes the stream."""
    L = lib()
    _bind_surrogate(L)
    p = _particles(pos, box, 1.0)
    g = _grid3(nc)
    ncube = int(pos.shape[0] * pos.shape[1] * pos.shape[2])
    if n_cubes is None:
        n_cubes = ncube - first_cube
    if capacity is None:
        capacity = 6 * n_cubes
    nbytes = C.c_size_t(0)
    _check(L.psd_surrogate_examples_workspace_size(n_cubes, C.byref(nbytes)),
           "psd_surrogate_examples_workspace_size")
    dev = pos.device
    ws = torch.empty(max(int(nbytes.value), 1), dtype=torch.uint8, device=dev)
    feat = torch.empty((capacity, 12), dtype=torch.float32, device=dev)
    frac = torch.empty((capacity, 8), dtype=torch.float64, device=dev)
    mask = torch.empty(capacity, dtype=torch.uint8, device=dev)
    ids = torch.empty(capacity, dtype=torch.int64, device=dev) if with_ids else None
    n_out = C.c_int64(0)
    ncs = (C.c_int32 * 3)(*g)
    _check(L.psd_surrogate_examples(pos.data_ptr(), C.byref(p), ncs, first_cube, n_cubes,
                                    min_cells, feat.data_ptr(), frac.data_ptr(), mask.data_ptr(),
                                    ids.data_ptr() if ids is not None else None, capacity,
                                    C.byref(n_out), ws.data_ptr(), ws.numel(),
                                    _stream_handle(stream)),
           "psd_surrogate_examples")
    n = min(int(n_out.value), capacity)
    out = {"feat": feat[:n], "frac": frac[:n], "mask": mask[:n], "found": int(n_out.value)}
    if ids is not None:
        out["tet"] = ids[:n]
    return out


def exact_fractions(tets: torch.Tensor, frac: torch.Tensor | None = None,
                    stream=None) -> torch.Tensor:
    """Exact overlap fractions [n, 8] (float64) of tetrahedra [n, 4, 3] (float32 vertices
    relative to the low corner of a 2x2x2 cell block, in [0, 2)) with the block's cells,
    cell c = 4 dx + 2 dy + dz; NaN rows for vertices outside the block."""
    L = lib()
    _bind_surrogate(L)
    _cuda(tets, torch.float32, (4, 3), "tets")
    n = int(tets.shape[0])
    if frac is None:
        frac = torch.empty((n, 8), dtype=torch.float64, device=tets.device)
    _cuda(frac, torch.float64, (8,), "frac")
    _check(L.psd_exact_fractions(tets.data_ptr(), frac.data_ptr(), n, _stream_handle(stream)),
           "psd_exact_fractions")
    return frac


def surrogate_forward(params: torch.Tensor, feat: torch.Tensor, mask: torch.Tensor,
                      probs: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Network probabilities [n, 8] for features [n, 12] and cell masks [n]."""
    L = lib()
    _bind_surrogate(L)
    _check_params(params)
    _cuda(feat, torch.float32, (12,), "feat")
    n = int(feat.shape[0])
    if mask.numel() != n or mask.dtype != torch.uint8 or not mask.is_cuda:
        raise ValueError("mask must be a CUDA uint8 tensor [n]")
    if probs is None:
        probs = torch.empty((n, 8), dtype=torch.float32, device=feat.device)
    _cuda(probs, torch.float32, (8,), "probs")
    _check(L.psd_surrogate_forward(params.data_ptr(), feat.data_ptr(), mask.data_ptr(), n,
                                   probs.data_ptr(), _stream_handle(stream)),
           "psd_surrogate_forward")
    return probs


def surrogate_backward(params: torch.Tensor, feat: torch.Tensor, frac: torch.Tensor,
                       mask: torch.Tensor, idx: torch.Tensor | None = None,
                       grad: torch.Tensor | None = None, loss: torch.Tensor | None = None,
                       stream=None):
    """(grad [9672] float32, loss [1] float64): gradient and value of the mean soft-label
    cross entropy over the batch idx (or all samples)."""
    L = lib()
    _bind_surrogate(L)
    _check_params(params)
    _cuda(feat, torch.float32, (12,), "feat")
    _cuda(frac, torch.float64, (8,), "frac")
    n = int(feat.shape[0]) if idx is None else int(idx.numel())
    if idx is not None and (idx.dtype != torch.int64 or not idx.is_cuda or not idx.is_contiguous()):
        raise ValueError("idx must be a contiguous CUDA int64 tensor")
    dev = feat.device
    if grad is None:
        grad = torch.empty(PSD_SURROGATE_PARAMS, dtype=torch.float32, device=dev)
    _check_params(grad)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float64, device=dev)
    _check(L.psd_surrogate_backward(params.data_ptr(), feat.data_ptr(), frac.data_ptr(),
                                    mask.data_ptr(), idx.data_ptr() if idx is not None else None,
                                    n, grad.data_ptr(), loss.data_ptr(), _stream_handle(stream)),
           "psd_surrogate_backward")
    return grad, loss


def surrogate_adam(params: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor,
                   step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
                   eps: float = 1e-8, stream=None) -> None:
    """One Adam update of params (in place) with moments m, v."""
    L = lib()
    _bind_surrogate(L)
    for t in (params, grad, m, v):
        _check_params(t)
    _check(L.psd_surrogate_adam(params.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(),
                                int(step), float(lr), float(beta1), float(beta2), float(eps),
                                _stream_handle(stream)),
           "psd_surrogate_adam")


def surrogate_train_steps(params: torch.Tensor, feat: torch.Tensor, frac: torch.Tensor,
                          mask: torch.Tensor, order: torch.Tensor, batch: int, lr: torch.Tensor,
                          m: torch.Tensor, v: torch.Tensor, step0: int, grad: torch.Tensor,
                          losses: torch.Tensor | None = None, beta1: float = 0.9,
                          beta2: float = 0.999, eps: float = 1e-8, stream=None) -> None:
    """len(lr) Adam steps in one launch: step s takes order[s*batch:(s+1)*batch], forms its
    gradient at the current params and updates params, m, v in place with step count
    step0 + s + 1 and rate lr[s]; losses[s] gets its mean loss.  grad is scratch."""
    L = lib()
    _bind_surrogate(L)
    for t in (params, m, v, grad):
        _check_params(t)
    _cuda(feat, torch.float32, (12,), "feat")
    _cuda(frac, torch.float64, (8,), "frac")
    for t, dt, name in ((order, torch.int64, "order"), (lr, torch.float32, "lr"),
                        (mask, torch.uint8, "mask")):
        if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous CUDA {dt} tensor")
    steps = int(lr.numel())
    if losses is not None and (losses.dtype != torch.float64 or not losses.is_cuda or
                               not losses.is_contiguous() or losses.numel() < steps):
        raise ValueError(f"losses must be a contiguous CUDA float64 tensor of {steps} values")
    _check(L.psd_surrogate_train_steps(params.data_ptr(), feat.data_ptr(), frac.data_ptr(),
                                       mask.data_ptr(), order.data_ptr(), int(order.numel()),
                                       int(batch), steps, int(step0), lr.data_ptr(), float(beta1),
                                       float(beta2), float(eps), m.data_ptr(), v.data_ptr(),
                                       grad.data_ptr(),
                                       losses.data_ptr() if losses is not None else None,
                                       _stream_handle(stream)),
           "psd_surrogate_train_steps")


def train_surrogate(params: torch.Tensor, feat: torch.Tensor, frac: torch.Tensor,
                    mask: torch.Tensor, order, batch: int = 4096, lr: float = 1e-3,
                    lr_final: float | None = None, state=None, stream=None,
                    steps_per_launch: int = 256) -> dict:
    """Adam over the examples, batches taken in the given sample order (a host or device
    int64 array; the last batch may be shorter).  The learning rate decays geometrically to
    lr_final over the run when given.  Up to steps_per_launch steps run in one launch
    (psd_surrogate_train_steps); steps_per_launch=0 makes every step one backward and one
    Adam launch.  Returns the optimizer state (m, v, step) with the per-step losses
    (device float64)."""
    dev = feat.device
    if state is None:
        state = {"m": torch.zeros_like(params), "v": torch.zeros_like(params), "step": 0}
    order_t = torch.as_tensor(order, dtype=torch.int64).to(dev).contiguous()
    n = int(order_t.numel())
    steps = (n + batch - 1) // batch
    losses = torch.empty(steps, dtype=torch.float64, device=dev)
    grad = torch.empty_like(params)
    decay = (lr_final / lr) ** (1.0 / max(steps - 1, 1)) if lr_final else 1.0
    rates = []
    rate = lr
    for _ in range(steps):
        rates.append(rate)
        rate *= decay
    if steps_per_launch > 0:
        rates_t = torch.tensor(rates, dtype=torch.float32).to(dev)
        for s0 in range(0, steps, steps_per_launch):
            k = min(steps_per_launch, steps - s0)
            surrogate_train_steps(params, feat, frac, mask, order_t[s0 * batch:], batch,
                                  rates_t[s0:s0 + k], state["m"], state["v"], state["step"], grad,
                                  losses=losses[s0:s0 + k], stream=stream)
            state["step"] += k
    else:
        for s in range(steps):
            sl = order_t[s * batch:(s + 1) * batch]
            surrogate_backward(params, feat, frac, mask, idx=sl, grad=grad, loss=losses[s:s + 1],
                               stream=stream)
            state["step"] += 1
            surrogate_adam(params, grad, state["m"], state["v"], state["step"], rates[s],
                           stream=stream)
    state["losses"] = losses
    return state


# ---------------------------------------------------------------------------
# Snapshot ingest and coarse octree levels
# ---------------------------------------------------------------------------

def _bind_extra(L):
    if getattr(L, "_extra_bound", False):
        return
    L.psd_reorder_workspace_size.restype = C.c_int
    L.psd_reorder_workspace_size.argtypes = [C.POINTER(C.c_int32), C.POINTER(C.c_size_t)]
    L.psd_reorder_by_id.restype = C.c_int
    L.psd_reorder_by_id.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64,
                                    C.POINTER(C.c_int32), C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_size_t, C.c_void_p]
    L.psd_octree_coarsen.restype = C.c_int
    L.psd_octree_coarsen.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_int32, C.c_int32,
                                     C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p]
    L._extra_bound = True


def reorder_workspace_size(np_) -> int:
    L = lib()
    _bind_extra(L)
    g = (C.c_int32 * 3)(*_grid3(np_))
    nbytes = C.c_size_t(0)
    _check(L.psd_reorder_workspace_size(g, C.byref(nbytes)), "psd_reorder_workspace_size")
    return int(nbytes.value)


def reorder_by_id(ids: torch.Tensor, pos_in: torch.Tensor, np_, id_base: int = 0,
                  out: torch.Tensor | None = None, check: torch.Tensor | None = None,
                  workspace: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Snapshot records (ids [n] int64, pos_in [n, 3] float32) placed on the Lagrangian grid
    [np0, np1, np2, 3]: slot ids[r] - id_base gets record r.  ``check`` (int64[3], optional)
    receives (ids out of range, duplicate slots, slots never named)."""
    L = lib()
    _bind_extra(L)
    g = _grid3(np_)
    if (not ids.is_cuda or ids.dtype != torch.int64 or ids.dim() != 1 or
            not ids.is_contiguous()):
        raise ValueError("ids must be a contiguous CUDA int64 tensor [n]")
    n = int(ids.numel())
    if (not pos_in.is_cuda or pos_in.dtype != torch.float32 or tuple(pos_in.shape) != (n, 3) or
            not pos_in.is_contiguous()):
        raise ValueError("pos_in must be a contiguous CUDA float32 tensor [n, 3]")
    shape = g + (3,)
    if out is None:
        out = torch.zeros(shape, dtype=torch.float32, device=pos_in.device)
    elif (out.dtype != torch.float32 or tuple(out.shape) != shape or not out.is_contiguous() or
          not out.is_cuda):
        raise ValueError(f"out must be a contiguous CUDA float32 tensor of shape {shape}")
    if check is not None:
        if (check.dtype != torch.int64 or not check.is_cuda or check.numel() < 3 or
                not check.is_contiguous()):
            raise ValueError("check must be a contiguous CUDA int64 tensor with 3 entries")
        workspace = _workspace(workspace, reorder_workspace_size(g), pos_in.device)
    npc = (C.c_int32 * 3)(*g)
    _check(L.psd_reorder_by_id(ids.data_ptr() if n else None, pos_in.data_ptr() if n else None, n,
                               int(id_base), npc, out.data_ptr(),
                               check.data_ptr() if check is not None else None,
                               workspace.data_ptr() if workspace is not None else None,
                               workspace.numel() * workspace.element_size()
                               if workspace is not None else 0,
                               _stream_handle(stream)),
           "psd_reorder_by_id")
    return out


def octree_coarsen(tree: "Octree", leaves: torch.Tensor, density: bool = False,
                   out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Every node's B^3 block [n_nodes, B, B, B] (node order): leaves copied, internal nodes
    as 2x2x2 sums of their children's cells (averages when ``density``)."""
    L = lib()
    _bind_extra(L)
    B = tree.block
    lshape = (tree.n_leaves, B, B, B)
    if (leaves.dtype != torch.float32 or tuple(leaves.shape) != lshape or
            not leaves.is_contiguous() or not leaves.is_cuda):
        raise ValueError(f"leaves must be a contiguous CUDA float32 tensor of shape {lshape}")
    shape = (tree.n_nodes, B, B, B)
    if out is None:
        out = torch.zeros(shape, dtype=torch.float32, device=leaves.device)
    elif (out.dtype != torch.float32 or tuple(out.shape) != shape or not out.is_contiguous() or
          not out.is_cuda):
        raise ValueError(f"out must be a contiguous CUDA float32 tensor of shape {shape}")
    _check(L.psd_octree_coarsen(tree.nodes.data_ptr(), tree.n_nodes, tree.n_leaves, B,
                                tree.max_level, leaves.data_ptr(), out.data_ptr(),
                                PSD_OUT_DENSITY if density else 0, _stream_handle(stream)),
           "psd_octree_coarsen")
    return out
