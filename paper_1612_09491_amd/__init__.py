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

STAT_NAMES = ("tets", "pairs", "clips_or_columns", "nonzero", "inverted", "degenerate")


class PsdError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__(f"{where}: {code} ({detail})")
        self.code = code


class Particles(C.Structure):
    _fields_ = [("np", C.c_int32 * 3), ("box", C.c_double), ("total_mass", C.c_double)]


class Options(C.Structure):
    _fields_ = [("flags", C.c_uint32), ("stats", C.c_void_p)]


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


def uniform_workspace_size(np_, nc, flags: int = 0, box: float = 1.0, mass: float = 1.0) -> int:
    p = Particles()
    for a, n in enumerate(_grid3(np_)):
        p.np[a] = n
    p.box, p.total_mass = float(box), float(mass)
    ncs = (C.c_int32 * 3)(*_grid3(nc))
    o = Options(flags, None)
    nbytes = C.c_size_t(0)
    _check(lib().psd_uniform_workspace_size(C.byref(p), ncs, C.byref(o), C.byref(nbytes)),
           "psd_uniform_workspace_size")
    return int(nbytes.value)


def deposit_uniform(pos: torch.Tensor, nc, box: float = 1.0, mass: float = 1.0, flags: int = 0,
                    out: torch.Tensor | None = None, mass_sum: torch.Tensor | None = None,
                    stats: torch.Tensor | None = None, workspace: torch.Tensor | None = None,
                    stream=None) -> torch.Tensor:
    """Cell masses (or densities with PSD_OUT_DENSITY) on a periodic nc grid.

    Returns ``out`` (float32, or float64 with PSD_PREC_FP64).  ``mass_sum``
    (float64[1]) receives the FP64 sum of deposited mass; ``stats`` (int64[8])
    receives counters (see STAT_NAMES).  Asynchronous on the current stream.
    """
    p = _particles(pos, box, mass)
    g = _grid3(nc)
    dtype = torch.float64 if flags & PSD_PREC_FP64 else torch.float32
    if out is None:
        out = torch.empty(g, dtype=dtype, device=pos.device)
    elif out.dtype != dtype or tuple(out.shape) != g or not out.is_contiguous() or not out.is_cuda:
        raise ValueError(f"out must be a contiguous CUDA {dtype} tensor of shape {g}")
    nbytes = uniform_workspace_size(tuple(pos.shape[:3]), g, flags, box, mass)
    if workspace is None:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=pos.device)
    if mass_sum is not None and (mass_sum.dtype != torch.float64 or not mass_sum.is_cuda):
        raise ValueError("mass_sum must be a CUDA float64 tensor")
    if stats is not None and (stats.dtype != torch.int64 or stats.numel() < 8 or not stats.is_cuda):
        raise ValueError("stats must be a CUDA int64 tensor with 8 entries")
    o = Options(flags, stats.data_ptr() if stats is not None else None)
    ncs = (C.c_int32 * 3)(*g)
    _check(lib().psd_deposit_uniform(pos.data_ptr(), C.byref(p), ncs, out.data_ptr(),
                                     mass_sum.data_ptr() if mass_sum is not None else None,
                                     C.byref(o), workspace.data_ptr(), workspace.numel(),
                                     _stream_handle(stream)),
           "psd_deposit_uniform")
    return out
