"""Benchmark: tetrahedra deposited per second on one MI355X.

Workload: 256^3 particles on a periodic unit box (Zel'dovich displacement,
rms 2 spacings, seed 2) -> 100,663,296 tetrahedra deposited exactly onto a
512^3 FP32 grid.  One step = one full psd_deposit_uniform call (output
zeroing, tetrahedron generation, cell walk, exact clipping, scatter, FP64 mass
sum) with the positions already resident in HBM.

Prints ONE JSON line.  Also reports:
  roofline      the deposit kernel's own algorithmic work (the cost model in
                costmodel.py, counted on a sample of the workload) per second
                against the chip's VALU issue rate, with the atomic and HBM
                terms beside it (atomic rates from the project's own
                microbenchmarks) and the paper's per-cell method as an
                equivalent rate;
  cpu_baseline  the FP64 oracle timed on a seeded sample of the same workload
                on the host cores (and on one thread), with the CPU model;
  surrogate     the learned-surrogate path in tets/s with its whole-grid
                density L1 against the oracle, on 256^3 -> 64^3 where most
                tetrahedra are eligible (and on the benchmark workload).
Secondary workloads (--workload): the adaptive octree, the 64-box batch, the
surrogate workload, and snapshot ingest (an HBM-bound scatter).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import subprocess
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "tetrahedra deposited/sec on 1 MI355X, exact vs surrogate at stated density L1 error"
WORKLOAD = "zel256_g512"

# VALU issue rate: 256 CUs x 64 lanes x 2.4 GHz (one lane-op per lane per clock:
# an FP64 or unpacked FP32 add, mul or FMA; packed FP32 is not used).
SIMDS = 256 * 4            # compute units x SIMDs, MI355X
CLOCK_HZ = 2.4e9           # peak engine clock
PEAK_VALU_OPS = 256 * 64 * CLOCK_HZ
PEAK_HBM = 8.0e12          # bytes/s, vendor figure

# Unit costs (lane-ops) of the paper's per-cell method, per counted event:
# tetrahedron setup, bbox-cell classification, signed distance per vertex per
# plane visit, edge cut, sub-tetrahedron volume, scatter of a non-zero deposit.
PAPER_COST = {"tet": 60, "pair": 24, "pv": 4, "cut": 9, "sub": 20, "nz": 2}


# Sources that define the deposit kernel; traffic counters taken on another
# version of them are not reported.
KERNEL_SOURCES = ("psd_cumulative.hip", "psd_device.h", "psd_internal.h")


def source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1612_09491_amd", "csrc")
    for name in KERNEL_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def paper_ops_per_tet(cnt: dict) -> float:
    n = max(cnt["n_tet"], 1)
    return (PAPER_COST["tet"] * cnt["n_tet"] + PAPER_COST["pair"] * cnt["n_pair"] +
            PAPER_COST["pv"] * cnt["n_pv"] + PAPER_COST["cut"] * cnt["n_cut"] +
            PAPER_COST["sub"] * cnt["n_sub"] + PAPER_COST["nz"] * cnt["n_nonzero"]) / n


def host_threads() -> int:
    return int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)


def cpu_info() -> dict:
    """CPU model and core counts of this host (lscpu)."""
    info = {"model": None, "sockets": None, "cores_per_socket": None, "logical_cpus": os.cpu_count()}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
    except (OSError, subprocess.SubprocessError):
        return info
    for line in txt.splitlines():
        k, _, v = line.partition(":")
        v = v.strip()
        if k.strip() == "Model name":
            info["model"] = v
        elif k.strip() == "Socket(s)":
            info["sockets"] = int(v) if v.isdigit() else v
        elif k.strip() == "Core(s) per socket":
            info["cores_per_socket"] = int(v) if v.isdigit() else v
    if isinstance(info["sockets"], int) and isinstance(info["cores_per_socket"], int):
        info["physical_cores"] = info["sockets"] * info["cores_per_socket"]
    return info


class ClockSampler:
    """Engine clock (MHz) read from rocm-smi while the timed loop runs."""

    def __init__(self, delay_s: float = 0.5):
        self.samples: list[float] = []
        self.error = None
        self._stop = threading.Event()
        self._t = threading.Thread(target=self._run, args=(delay_s,), daemon=True)

    def _read(self):
        try:
            txt = subprocess.run(["rocm-smi", "--showclocks"], capture_output=True, text=True,
                                 timeout=20).stdout
        except (OSError, subprocess.SubprocessError) as e:
            self.error = str(e)
            return None
        m = re.search(r"sclk clock level:\s*\d+:\s*\((\d+(?:\.\d+)?)\s*Mhz\)", txt, re.I)
        return float(m.group(1)) if m else None

    def _run(self, delay_s):
        if self._stop.wait(delay_s):
            return
        while not self._stop.is_set():
            v = self._read()
            if v is not None:
                self.samples.append(v)
            elif self.error is None:
                self.error = "no sclk line in rocm-smi output"
            if self._stop.wait(1.0):
                return

    def __enter__(self):
        self._t.start()
        return self

    def __exit__(self, *exc):
        self._stop.set()
        self._t.join(timeout=30)

    def summary(self) -> dict:
        if not self.samples:
            return {"sclk_mhz": None, "source": "rocm-smi --showclocks", "error": self.error}
        s = sorted(self.samples)
        return {"sclk_mhz": s[len(s) // 2], "sclk_mhz_min": s[0], "sclk_mhz_max": s[-1],
                "samples": len(s), "source": "rocm-smi --showclocks during the timed loop"}


def atomic_peaks(torch) -> dict:
    """Rates of the operations the deposit's scatter and level walk use, from the
    project's microbenchmarks (libpsd_peaks.so), timed with events on one stream."""
    import ctypes as C
    from paper_1612_09491_amd import build as hip_build
    if not os.path.exists(hip_build.PEAKS_LIB):
        return {"error": f"{hip_build.PEAKS_LIB} is missing"}
    L = C.CDLL(hip_build.PEAKS_LIB)
    L.peaks_global_atomic_f32.restype = C.c_int64
    L.peaks_global_atomic_f32.argtypes = [C.c_void_p, C.c_int64, C.c_int, C.c_int, C.c_int,
                                          C.c_void_p]
    L.peaks_lds_atomic.restype = C.c_int64
    L.peaks_lds_atomic.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p]
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        n = 0
        for _ in range(reps):
            n += fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return n / (e0.elapsed_time(e1) / 1e3)

    words = 1 << 27  # 512 MiB of FP32, beyond the last-level caches
    buf = torch.zeros(words, dtype=torch.float32, device=dev)
    blocks = 256 * 16
    out = {}
    for name, pat in (("global_atomic_add_f32_coalesced", 0), ("global_atomic_add_f32_random", 1),
                      ("global_atomic_add_f32_column_walks", 2),
                      ("global_atomic_add_f32_tile_rows", 3)):
        def run(pat=pat):
            n = L.peaks_global_atomic_f32(buf.data_ptr(), words, blocks, 64, pat, sh)
            if n < 0:
                raise RuntimeError("peaks_global_atomic_f32 refused its arguments")
            return n
        out[name] = timed(run)
    del buf
    lds_out = torch.zeros(blocks * 256, dtype=torch.float64, device=dev)
    for name, f64 in (("ds_add_f32", 0), ("ds_add_f64", 1)):
        def run(f64=f64):
            n = L.peaks_lds_atomic(lds_out.data_ptr(), blocks, 1024, f64, sh)
            if n < 0:
                raise RuntimeError("peaks_lds_atomic refused its arguments")
            return n
        out[name] = timed(run)
    # plain device copy: bytes read + written per second
    src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)

    def copy():
        dst.copy_(src)
        return 2 * src.numel() * 4
    out["copy_bytes_per_s"] = timed(copy)
    del src, dst
    out["unit"] = "operations/s (copy: bytes/s)"
    return out


def cpu_baseline(pos: np.ndarray, nc: int, gpu_grid: np.ndarray | None, n_cubes: int,
                 seed: int = 12345, other_grids: dict | None = None,
                 single_thread_cubes: int = 0) -> dict:
    """The FP64 oracle on a seeded random sample of Lagrangian cubes, on host cores."""
    import oracle
    oracle.build_oracle(force=False)
    npart = pos.shape[0]
    rng = np.random.default_rng(seed)
    cubes = np.sort(rng.choice(npart ** 3, size=n_cubes, replace=False)).astype(np.int64)
    threads = host_threads()
    t0 = time.perf_counter()
    _, cnt = oracle.deposit_uniform(pos, nc, cubes=cubes, mode=oracle.TRIVIAL, nthreads=threads)
    dt = time.perf_counter() - t0
    # counting pass with the paper's own splitting scheme (not timed)
    _, pcnt = oracle.deposit_uniform(pos, nc, cubes=cubes, mode=oracle.TRIVIAL | oracle.PAPER,
                                     nthreads=threads)
    out = {
        "value": 6 * n_cubes / dt,
        "unit": "tets/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{n_cubes} random Lagrangian cubes ({6 * n_cubes} tets) of the workload, "
                  f"seed {seed}, FP64 polytope clipper, {dt:.1f} s on {threads} threads",
        "host": cpu_info(),
        "counters_per_tet": {k: v / max(pcnt["n_tet"], 1) for k, v in pcnt.items()},
    }
    if single_thread_cubes:
        sub = cubes[:: max(1, n_cubes // single_thread_cubes)][:single_thread_cubes]
        t0 = time.perf_counter()
        oracle.deposit_uniform(pos, nc, cubes=sub, mode=oracle.TRIVIAL, nthreads=1)
        d1 = time.perf_counter() - t0
        out["single_thread"] = {"value": 6 * len(sub) / d1, "unit": "tets/s", "cores": 1,
                                "sample": f"{len(sub)} of the same cubes, {d1:.1f} s"}
    if gpu_grid is not None:
        # sampled-block density error of the GPU grid against the oracle
        blo = [int(x) for x in np.random.default_rng(seed + 1).integers(0, nc - 16, size=3)]
        ref, _ = oracle.deposit_uniform(pos, nc, region=(blo, (16, 16, 16)), nthreads=threads)
        blk = gpu_grid[blo[0]:blo[0] + 16, blo[1]:blo[1] + 16, blo[2]:blo[2] + 16]
        out["gpu_block_l1"] = float(np.abs(blk - ref).sum() / np.abs(ref).sum())
        out["gpu_block"] = blo
        for name, g in (other_grids or {}).items():
            b2 = g[blo[0]:blo[0] + 16, blo[1]:blo[1] + 16, blo[2]:blo[2] + 16]
            out[f"{name}_block_l1"] = float(np.abs(b2 - ref).sum() / np.abs(ref).sum())
    out["_paper_counters"] = pcnt
    out["_counters"] = cnt
    return out


def own_work(pos: np.ndarray, nc, n_cubes: int, cap: int, nz_per_tet: float,
             seed: int = 12346) -> dict:
    """Own-work lane operations per tetrahedron of the cumulative kernel (costmodel.py's
    frozen unit costs) from a CPU replay of its walk on a seeded cube sample."""
    import costmodel
    npart = pos.shape[0] * pos.shape[1] * pos.shape[2]
    rng = np.random.default_rng(seed)
    cubes = np.sort(rng.choice(npart, size=min(n_cubes, npart), replace=False))
    t0 = time.perf_counter()
    ev = costmodel.count_events(pos, nc, cubes, cap=cap)
    dt = time.perf_counter() - t0
    n = max(ev["tets_sampled"], 1)
    per = {k: ev[k] / n for k in costmodel.EVENTS}
    per["nz"] = nz_per_tet
    ops = sum(costmodel.COST[k] * per[k] for k in costmodel.COST)
    return {"ops_per_tet": ops, "events_per_tet": per, "unit_costs": dict(costmodel.COST),
            "sample": f"{len(cubes)} random Lagrangian cubes, CPU replay of the walk "
                      f"({dt:.1f} s); non-zero deposits per tet from the oracle sample"}


# template arguments after the buffer size of each deposit-kernel instance:
# tets set up at once, tiles per batch, work counters, ring size, slab form
GROUP_OF_CAP = {512: "16, 16, false, 0, false", 960: "32, 16, false, 0, false",
                1024: "8, 8, false, 128, false", 1408: "8, 8, false, 0, false",
                2048: "32, 32, false, 0, false"}

SURROGATE_WEIGHTS = os.path.join(ROOT, "paper_1612_09491_amd", "surrogate_zel256_g64.npy")


def time_deposit(psd, torch, pt, nc, flags, reps, surrogate=None, out=None, ws=None):
    """Mean wall time (ms) of `reps` deposits after one warm-up, and the last grid."""
    stream = torch.cuda.current_stream()
    dtype = torch.float64 if flags & psd.PSD_PREC_FP64 else torch.float32
    if out is None:
        out = torch.empty((nc, nc, nc), dtype=dtype, device=pt.device)
    if ws is None:
        ws = torch.empty(psd.uniform_workspace_size(tuple(pt.shape[:3]), nc, flags),
                         dtype=torch.uint8, device=pt.device)
    psd.deposit_uniform(pt, nc, flags=flags, out=out, workspace=ws, stream=stream, surrogate=surrogate)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        psd.deposit_uniform(pt, nc, flags=flags, out=out, workspace=ws, stream=stream,
                            surrogate=surrogate)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps, out


def rel_l1(a, b) -> float:
    return float((a - b).abs().sum().item() / b.abs().sum().item())


def np_rel_l1(a, b) -> float:
    return float(np.abs(a - b).sum() / np.abs(b).sum())


def np_rel_linf(a, b) -> float:
    return float(np.abs(a - b).max() / np.abs(b).max())


def oracle_grid(pos: np.ndarray, nc: int) -> tuple[np.ndarray, float]:
    """The oracle's whole grid (host threads) and its wall time in seconds."""
    import oracle
    oracle.build_oracle(force=False)
    t0 = time.perf_counter()
    ref, _ = oracle.deposit_uniform(pos, nc, mode=oracle.TRIVIAL, nthreads=host_threads())
    return ref, time.perf_counter() - t0


def surrogate_g64(psd, torch, reps: int, with_oracle: bool) -> dict:
    """256^3 -> 64^3 (0.25 cells per spacing, ~72% of tets eligible): exact and surrogate
    paths on the same positions, each grid's density L1 against the oracle's whole grid."""
    from synth import workload
    dev = torch.device("cuda:0")
    pos, p = workload("zel256_g64")
    nc = p["nc"]
    ntet = 6 * p["np"] ** 3
    pt = torch.from_numpy(pos).to(dev)
    w = torch.from_numpy(np.load(SURROGATE_WEIGHTS).astype(np.float32)).to(dev)
    ms_x, g_x = time_deposit(psd, torch, pt, nc, 0, reps)
    ms_s, g_s = time_deposit(psd, torch, pt, nc, psd.PSD_SURROGATE, reps, surrogate=w)
    st = torch.zeros(8, dtype=torch.int64, device=dev)
    psd.deposit_uniform(pt, nc, flags=psd.PSD_SURROGATE, stats=st, surrogate=w)
    torch.cuda.synchronize()
    gx, gs = g_x.double().cpu().numpy(), g_s.double().cpu().numpy()
    out = {"workload": "zel256_g64", "tets": ntet, "grid": [nc, nc, nc],
           "exact_tets_per_s": ntet / (ms_x / 1e3), "exact_ms": ms_x,
           "surrogate_tets_per_s": ntet / (ms_s / 1e3), "surrogate_ms": ms_s,
           "speedup": ms_x / ms_s, "eligible_tets": int(st[6].item()),
           "density_l1_vs_exact": np_rel_l1(gs, gx)}
    if with_oracle:
        ref, dt = oracle_grid(pos, nc)
        out["density_l1_vs_oracle"] = np_rel_l1(gs, ref)
        out["density_linf_vs_oracle"] = np_rel_linf(gs, ref)
        out["exact_density_l1_vs_oracle"] = np_rel_l1(gx, ref)
        out["oracle_grid"] = f"whole 64^3 grid, {dt:.1f} s on {host_threads()} host threads"
    return out


def load_traffic(kernel: str, workload: str) -> dict | None:
    """HBM bytes per launch from committed rocprofv3 --pmc summaries, if current."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_hash") != source_hash():
        return None
    return t


def oracle_sample_counts(boxes, n_cubes_total: int, seed: int, nc_of) -> dict:
    """Oracle on a seeded cube sample spread over boxes in proportion to their cubes:
    wall time of the exact deposit (host cores) and the paper-scheme work counters."""
    import oracle
    oracle.build_oracle(force=False)
    threads = host_threads()
    rng = np.random.default_rng(seed)
    total = sum(b.shape[0] * b.shape[1] * b.shape[2] for b in boxes)
    dt, tets = 0.0, 0
    pc = None
    nz = 0.0
    for i, pos in enumerate(boxes):
        nb = pos.shape[0] * pos.shape[1] * pos.shape[2]
        k = max(16, int(round(n_cubes_total * nb / total)))
        k = min(k, nb)
        cubes = np.sort(rng.choice(nb, size=k, replace=False)).astype(np.int64)
        t0 = time.perf_counter()
        _, c0 = oracle.deposit_uniform(pos, nc_of(i), cubes=cubes, mode=oracle.TRIVIAL,
                                       nthreads=threads)
        dt += time.perf_counter() - t0
        tets += 6 * k
        _, c = oracle.deposit_uniform(pos, nc_of(i), cubes=cubes,
                                      mode=oracle.TRIVIAL | oracle.PAPER, nthreads=threads)
        # weight each box's counters by its share of all tetrahedra
        w = nb / total / (6 * k)
        pc = {key: (pc[key] if pc else 0.0) + v * w for key, v in c.items()}
        nz += c0["n_nonzero"] * w
    return {"seconds": dt, "tets": tets, "threads": threads, "nz_per_tet": nz,
            "paper_ops_per_tet": paper_ops_per_tet({k: v for k, v in pc.items()} | {"n_tet": 1.0})}


def roofline_line(kernel: str, kernel_ms: float, ntet: int, own: dict | None,
                  paper_ops: float | None, n_atomic: float | None, hbm_bytes: float,
                  peaks: dict | None, clock: dict | None, traffic: dict | None) -> dict:
    """The dominant kernel against the VALU issue rate on its own algorithmic work, with the
    atomic and HBM terms: t_roof = max(ops / P_valu, atomics / P_atomic, bytes / P_hbm)."""
    t = kernel_ms / 1e3
    line = {"bound": "alu", "peak": PEAK_VALU_OPS / 1e12, "unit": "Top/s", "kernel": kernel,
            "kernel_ms": kernel_ms, "traffic": traffic["bytes_per_launch"] if traffic else None}
    terms = {}
    if own is not None:
        ops = own["ops_per_tet"] * ntet
        line["achieved"] = ops / t / 1e12
        line["frac"] = ops / t / PEAK_VALU_OPS
        line["own_ops_per_tet"] = own["ops_per_tet"]
        line["own_work"] = own
        terms["valu_s"] = ops / PEAK_VALU_OPS
        if clock and clock.get("sclk_mhz"):
            p_clk = 256 * 64 * clock["sclk_mhz"] * 1e6
            line["frac_at_measured_clock"] = ops / t / p_clk
    if paper_ops is not None:
        line["paper_method_equivalent"] = {
            "ops_per_tet": paper_ops, "rate_Top_s": paper_ops * ntet / t / 1e12,
            "equivalent_frac": paper_ops * ntet / t / PEAK_VALU_OPS,
            "note": "the paper's per-cell splitting priced with its frozen unit costs: the "
                    "work that method would do at this speed, not a fraction of a roofline"}
    if n_atomic is not None and peaks and "global_atomic_add_f32_tile_rows" in peaks:
        # the deposit's scatter: the lanes hold a tile's columns row by row (neighbouring
        # cells along one grid axis), each walking its column's levels along another
        pa = peaks["global_atomic_add_f32_tile_rows"]
        terms["atomic_s"] = n_atomic / pa
        line["atomic"] = {"n_atomic": n_atomic, "peak_tile_rows": pa,
                          "peak_column_walks": peaks.get("global_atomic_add_f32_column_walks"),
                          "peak_random": peaks.get("global_atomic_add_f32_random"),
                          "peak_coalesced": peaks.get("global_atomic_add_f32_coalesced"),
                          "achieved": n_atomic / t, "frac": n_atomic / t / pa,
                          "unit": "atomics/s"}
    terms["hbm_s"] = hbm_bytes / PEAK_HBM
    line["hbm"] = {"algorithmic_bytes": hbm_bytes, "achieved_GBps": hbm_bytes / t / 1e9,
                   "frac": hbm_bytes / t / PEAK_HBM}
    if terms:
        name = max(terms, key=terms.get)
        line["binding_term"] = name[:-2]
        line["frac_of_max_term"] = terms[name] / t
        line["terms_s"] = terms
    if traffic and traffic.get("valu_insts_per_launch"):
        # machine view of the same launch: wave64 VALU instructions (rocprofv3
        # SQ_INSTS_VALU of this kernel version) x 4 clocks over 1024 SIMDs, and the
        # share of lanes active per VALU instruction (VALUUtilization)
        line["valu_issue_frac"] = 4.0 * traffic["valu_insts_per_launch"] / (SIMDS * CLOCK_HZ * t)
        if traffic.get("valu_utilization_pct") is not None:
            line["valu_lanes_active_frac"] = traffic["valu_utilization_pct"] / 100.0
    return line


def events_loop(torch, stream, step, steps: int) -> tuple[float, float]:
    """(wall ms per step, event ms per step on the launch stream) of `steps` calls."""
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    return wall, e0.elapsed_time(e1) / steps


def bench_octree(args, torch, psd) -> dict:
    """Adaptive octree: 512^3 particles with clumps, 16^3-cell leaves, <= 4 levels."""
    from synth import workload
    dev = torch.device("cuda:0")
    print("generating 512^3 + clumps ...", file=sys.stderr, flush=True)
    pos, p = workload("clump512_octree")
    ntet = 6 * p["np"] ** 3
    pt = torch.from_numpy(pos).to(dev)
    stream = torch.cuda.current_stream()
    kw = dict(block=p["block"], max_level=p["max_level"], subblock=8, threshold=p["threshold"])
    tree = psd.build_octree(pt, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        tree = psd.build_octree(pt, **kw)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3 / 3
    nodes = tree.to_numpy()
    levels = np.bincount(nodes["level"][nodes["leaf_id"] >= 0], minlength=p["max_level"] + 1)
    out = torch.empty((tree.n_leaves, 16, 16, 16), dtype=torch.float32, device=dev)
    ms = torch.zeros(1, dtype=torch.float64, device=dev)
    ws = torch.empty(psd.octree_workspace_size(tuple(pos.shape[:3]), **kw), dtype=torch.uint8,
                     device=dev)
    flags = psd.PSD_OUT_DENSITY

    def step():
        psd.deposit_octree(pt, tree, flags=flags, out=out, mass_sum=ms, workspace=ws, stream=stream)

    for _ in range(args.warmup):
        step()
    ms_per_step, kernel_ms = events_loop(torch, stream, step, args.steps)
    # coarse levels of the internal nodes from the leaves (HBM-bound)
    coarse = torch.empty((tree.n_nodes, 16, 16, 16), dtype=torch.float32, device=dev)
    psd.octree_coarsen(tree, out, density=True, out=coarse)
    _, coarsen_ms = events_loop(torch, stream,
                                lambda: psd.octree_coarsen(tree, out, density=True, out=coarse), 5)
    coarsen_bytes = 4 * 16 ** 3 * (tree.n_leaves + tree.n_nodes + 8 * (tree.n_nodes - tree.n_leaves))
    finest = int(np.nonzero(levels)[0].max())
    nc_f = p["block"] << finest
    line = {"value": ntet / (ms_per_step / 1e3), "ms_per_step": ms_per_step,
            "dtype": "f64",
            "config": {"workload": "clump512_octree", "particles": p["np"] ** 3, "tets": ntet,
                       "leaves": tree.n_leaves, "nodes": tree.n_nodes,
                       "leaves_per_level": levels.tolist(), "block": p["block"],
                       "threshold": p["threshold"], "build_octree_ms": build_ms,
                       "path": "exact cumulative clipping in FP64 into 16^3 FP32 density leaves"},
            "mass_error": abs(float(ms.item()) - 1.0),
            "coarsen": {"ms": coarsen_ms, "bytes": coarsen_bytes,
                        "GBps": coarsen_bytes / (coarsen_ms / 1e3) / 1e9,
                        "hbm_frac": coarsen_bytes / (coarsen_ms / 1e3) / PEAK_HBM}}
    if not args.no_cpu:
        # the finest level's cells as a uniform grid carry the same algorithmic work
        o = oracle_sample_counts([pos], args.cpu_cubes, 12345, lambda i: nc_f)
        line["cpu_baseline"] = {"value": o["tets"] / o["seconds"], "unit": "tets/s",
                                "cores": o["threads"], "kind": "oracle", "host": cpu_info(),
                                "sample": f"{o['tets'] // 6} random Lagrangian cubes deposited "
                                          f"onto the finest level's {nc_f}^3 cells, "
                                          f"{o['seconds']:.1f} s"}
        own = own_work(pos, nc_f, args.model_cubes, 960, o["nz_per_tet"])
        line["roofline"] = roofline_line("queue_kernel<float, 960, 32, 16, false, 0, false>", kernel_ms, ntet, own,
                                         o["paper_ops_per_tet"], o["nz_per_tet"] * ntet,
                                         12.0 * pos.shape[0] ** 3 + out.numel() * 4.0,
                                         None, None, None)
    return line


def bench_batched(args, torch, psd) -> dict:
    """64 independent boxes of uneven size in one persistent launch, autotuned."""
    from synth import batched_box_specs, zeldovich_positions
    dev = torch.device("cuda:0")
    specs = batched_box_specs()
    print("generating 64 boxes ...", file=sys.stderr, flush=True)
    host = [zeldovich_positions(sp["np"], sp["rms"], sp["seed"]) for sp in specs]
    ntet = sum(6 * sp["np"] ** 3 for sp in specs)
    boxes = [(torch.from_numpy(h).to(dev), sp["nc"]) for h, sp in zip(host, specs)]
    t0 = time.perf_counter()
    best, best_ms = psd.autotune_batched(boxes)
    tune_s = time.perf_counter() - t0
    outs = [torch.empty((sp["nc"],) * 3, dtype=torch.float32, device=dev) for sp in specs]
    full = [(b[0], b[1], o) for b, o in zip(boxes, outs)]
    ms = torch.zeros(len(specs), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        psd.deposit_batched(full, mass_sums=ms, tuning=best, stream=stream)

    for _ in range(args.warmup):
        step()
    ms_per_step, kernel_ms = events_loop(torch, stream, step, args.steps)
    line = {"value": ntet / (ms_per_step / 1e3), "ms_per_step": ms_per_step, "dtype": "f64",
            "config": {"workload": "batched64", "boxes": len(specs), "tets": ntet,
                       "particles_per_box": [sp["np"] for sp in specs],
                       "tuning": {"lds_cap": best[0], "waves_per_cu": best[1],
                                  "ordered": best[2]},
                       "autotune_s": tune_s,
                       "path": "one persistent launch over 64 box descriptors, exact FP64"},
            "mass_error": float((ms - 1.0).abs().max().item())}
    if not args.no_cpu:
        o = oracle_sample_counts(host, args.cpu_cubes, 12345, lambda i: specs[i]["nc"])
        line["cpu_baseline"] = {"value": o["tets"] / o["seconds"], "unit": "tets/s",
                                "cores": o["threads"], "kind": "oracle", "host": cpu_info(),
                                "sample": f"{o['tets'] // 6} random Lagrangian cubes spread over "
                                          f"the 64 boxes by size, {o['seconds']:.1f} s"}
        # own work: the replay on each box's share of the sample, weighted by its tets
        import costmodel
        tot_ops, tot_w = 0.0, 0.0
        rng = np.random.default_rng(12346)
        for h, sp in zip(host, specs):
            k = max(8, args.model_cubes * sp["np"] ** 3 // sum(s["np"] ** 3 for s in specs))
            cubes = np.sort(rng.choice(sp["np"] ** 3, size=min(k, sp["np"] ** 3), replace=False))
            ev = costmodel.count_events(h, sp["nc"], cubes, cap=best[0])
            per_tet = costmodel.own_ops(ev) / max(ev["tets_sampled"], 1)
            tot_ops += per_tet * 6 * sp["np"] ** 3
            tot_w += 6 * sp["np"] ** 3
        own = {"ops_per_tet": tot_ops / tot_w + costmodel.COST["nz"] * o["nz_per_tet"],
               "sample": "CPU replay of the walk on a cube sample of every box"}
        line["roofline"] = roofline_line(f"queue_kernel<float, {best[0]}, {GROUP_OF_CAP[best[0]]}>",
                                         kernel_ms, ntet, own, o["paper_ops_per_tet"],
                                         o["nz_per_tet"] * ntet,
                                         sum(12.0 * sp["np"] ** 3 + 4.0 * sp["nc"] ** 3
                                             for sp in specs), None, None, None)
    return line


def bench_surrogate_workload(args, torch, psd) -> dict:
    """256^3 -> 64^3 (0.25 cells per spacing, ~72% of tets eligible for the network):
    the exact path and the surrogate path on the same positions."""
    if not os.path.exists(SURROGATE_WEIGHTS):
        raise SystemExit(f"{SURROGATE_WEIGHTS} is missing: train with paper_1612_09491_amd/train.py")
    s = surrogate_g64(psd, torch, max(1, args.steps), with_oracle=not args.no_cpu)
    line = {"value": s["surrogate_tets_per_s"], "ms_per_step": s["surrogate_ms"],
            "dtype": "bf16+f64",
            "config": {"workload": "zel256_g64", "particles": 256 ** 3, "tets": s["tets"],
                       "grid": s["grid"], "rms_displacement_spacings": 2.0, "seed": 6,
                       "weights": os.path.basename(SURROGATE_WEIGHTS),
                       "path": "learned surrogate (BF16 MFMA) for tets within 2x2x2 cells, "
                               "exact FP64 for the others"},
            "surrogate": s}
    if not args.no_cpu:
        from synth import workload
        pos, p = workload("zel256_g64")
        o = oracle_sample_counts([pos], args.cpu_cubes, 12345, lambda i: p["nc"])
        line["cpu_baseline"] = {"value": o["tets"] / o["seconds"], "unit": "tets/s",
                                "cores": o["threads"], "kind": "oracle", "host": cpu_info(),
                                "sample": f"{o['tets'] // 6} random Lagrangian cubes, exact FP64 "
                                          f"polytope clipper, {o['seconds']:.1f} s"}
    return line


def bench_ingest(args, torch, psd) -> dict:
    """Snapshot ingest: the benchmark's 256^3 records in a seeded random order scattered to
    their Lagrangian slots by ID, with the duplicate / missing check (HBM-bound)."""
    from synth import workload
    dev = torch.device("cuda:0")
    pos, p = workload(WORKLOAD)
    n = pos.shape[0] ** 3
    perm = np.random.default_rng(86).permutation(n)
    ids = torch.from_numpy(perm.astype(np.int64)).to(dev)
    rec = torch.from_numpy(np.ascontiguousarray(pos.reshape(-1, 3)[perm])).to(dev)
    out = torch.empty(pos.shape, dtype=torch.float32, device=dev)
    chk = torch.zeros(3, dtype=torch.int64, device=dev)
    ws = torch.empty(psd.reorder_workspace_size(pos.shape[:3]), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        psd.reorder_by_id(ids, rec, pos.shape[:3], out=out, check=chk, workspace=ws, stream=stream)

    for _ in range(max(1, args.warmup)):
        step()
    ms_per_step, kernel_ms = events_loop(torch, stream, step, max(args.steps, 5))
    ok = bool(torch.equal(out.cpu(), torch.from_numpy(pos))) and chk.cpu().tolist() == [0, 0, 0]
    # bytes: ids and records read, positions written, the occupancy map cleared, set
    # (one word read-modify-write per record) and counted
    words = (n + 31) // 32
    nbytes = n * (8 + 12 + 12) + words * 4 * 2 + n * 8
    line = {"metric": "particles placed/sec (snapshot ingest)", "unit": "particles/s",
            "value": n / (ms_per_step / 1e3), "ms_per_step": ms_per_step, "dtype": "u8",
            "config": {"workload": "ingest256", "records": n, "check": True,
                       "path": "scatter by Lagrangian ID with the occupancy check"},
            "restores_grid": ok,
            "roofline": {"bound": "hbm", "achieved": nbytes / (kernel_ms / 1e3) / 1e9,
                         "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                         "frac": nbytes / (kernel_ms / 1e3) / PEAK_HBM, "traffic": None,
                         "algorithmic_bytes": nbytes, "kernel_ms": kernel_ms,
                         "kernel": "scatter_by_id_kernel<true> + fill + missing_slots_kernel"}}
    return line


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-cubes", type=int, default=None,
                    help="Lagrangian cubes in the oracle's timed sample (default per workload, "
                         "about 10-30 s of host work)")
    ap.add_argument("--model-cubes", type=int, default=4000,
                    help="Lagrangian cubes of the own-work cost model's CPU replay")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the CPU baseline, the cost model and the oracle grids")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate leg")
    ap.add_argument("--no-cell", action="store_true",
                    help="skip the per-cell (cell-local FP32) method's timing")
    ap.add_argument("--workload", default=WORKLOAD,
                    choices=[WORKLOAD, "clump512_octree", "batched64", "zel256_g64", "ingest256"],
                    help="the benchmark workload (default) or a secondary one")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 256 MiB device copy, whose FETCH_SIZE and "
                         "WRITE_SIZE counters scale the deposit kernel's")
    args = ap.parse_args()
    if args.cpu_cubes is None:
        args.cpu_cubes = {"clump512_octree": 1_000_000, "zel256_g64": 1_500_000}.get(
            args.workload, 150_000)
    if args.gpus != 1:
        print(f"bench.py: the deposit runs on one GPU only (asked for --gpus {args.gpus}); "
              "sharding across GPUs is not implemented.", file=sys.stderr)
        return 2

    import torch
    import paper_1612_09491_amd as psd
    from synth import workload

    if not os.path.exists(psd.LIB_PATH):
        raise SystemExit(f"{psd.LIB_PATH} is missing: run __graft_entry__.build() first")

    if args.workload != WORKLOAD:
        fn = {"clump512_octree": bench_octree, "batched64": bench_batched,
              "zel256_g64": bench_surrogate_workload, "ingest256": bench_ingest}[args.workload]
        extra = fn(args, torch, psd)
        line = {"metric": METRIC, "unit": "tets/s", "n_gpus": 1, "steps": args.steps,
                "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
                "vs_baseline": None, "data": "synthetic"}
        line.update(extra)
        print(json.dumps(line), flush=True)
        return 0

    dev = torch.device("cuda:0")
    pos, p = workload(WORKLOAD)
    nc = p["nc"]
    ntet = 6 * p["np"] ** 3
    pt = torch.from_numpy(pos).to(dev)
    out = torch.empty((nc, nc, nc), dtype=torch.float32, device=dev)
    msum = torch.zeros(1, dtype=torch.float64, device=dev)
    ws = torch.empty(psd.uniform_workspace_size(pos.shape[:3], nc), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        psd.deposit_uniform(pt, nc, out=out, mass_sum=msum, workspace=ws, stream=stream)

    for _ in range(args.warmup):
        step()
    print(f"timing {args.steps} steps ...", file=sys.stderr, flush=True)
    # the timed region: K steps between synchronizations, bracketed by events on the
    # launch stream (the deposit kernel plus the grid fill, ~0.1 ms, and a counter reset)
    with ClockSampler() as clk:
        ms_per_step, kernel_ms = events_loop(torch, stream, step, args.steps)
    value = ntet / (ms_per_step / 1e3)
    mass_err = abs(float(msum.item()) - 1.0)
    grid = out.double().cpu().numpy()

    scratch = torch.zeros_like(out)
    st = torch.zeros(16, dtype=torch.int64, device=dev)
    psd.deposit_uniform(pt, nc, out=scratch, stats=st, workspace=ws, stream=stream,
                        flags=psd.PSD_WORK_COUNTERS)
    torch.cuda.synchronize()
    s = [int(x) for x in st.cpu().numpy()]
    gstats = dict(zip(psd.STAT_NAMES, s[:8]))
    gwork = {"column": s[2], "xpiece": s[8], "piece": s[9], "level": s[10], "colcell": s[11],
             "nz": s[3]}
    del scratch
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    print("FP64 grid, per-cell method, surrogate ...", file=sys.stderr, flush=True)
    # the same deposit into an FP64 grid (identical arithmetic, double atomics)
    ms64, _ = time_deposit(psd, torch, pt, nc, psd.PSD_PREC_FP64, reps=max(1, min(args.steps, 2)))
    # the per-cell method: cell-local FP32 clipping (one timed run), and the cached slab
    # clipping in FP32 beside it at the same error
    ms_cell, cell_grid = (None, None)
    ms_slab, slab_grid = (None, None)
    if not args.no_cell:
        ms_cell, g = time_deposit(psd, torch, pt, nc, psd.PSD_METHOD_CELL, reps=1)
        cell_grid = g.double().cpu().numpy()
        del g
        ms_slab, g = time_deposit(psd, torch, pt, nc, psd.PSD_METHOD_SLAB, reps=2)
        slab_grid = g.double().cpu().numpy()
        del g

    sur = None
    if not args.no_surrogate and os.path.exists(SURROGATE_WEIGHTS):
        w = torch.from_numpy(np.load(SURROGATE_WEIGHTS).astype(np.float32)).to(dev)
        ms_s, g_s = time_deposit(psd, torch, pt, nc, psd.PSD_SURROGATE,
                                 max(1, min(args.steps, 3)), surrogate=w)
        st8 = torch.zeros(8, dtype=torch.int64, device=dev)
        psd.deposit_uniform(pt, nc, flags=psd.PSD_SURROGATE, stats=st8, surrogate=w)
        sur = {"weights": os.path.basename(SURROGATE_WEIGHTS),
               WORKLOAD: {"tets_per_s": ntet / (ms_s / 1e3), "ms": ms_s,
                          "eligible_tets": int(st8[6].item()),
                          "density_l1_vs_exact": rel_l1(g_s.double(), out.double())}}
        del g_s
        sur["zel256_g64"] = surrogate_g64(psd, torch, max(1, min(args.steps, 3)),
                                          with_oracle=not args.no_cpu)

    peaks = None
    try:
        peaks = atomic_peaks(torch)
    except Exception as e:  # measurement aid: report and go on
        peaks = {"error": str(e)}

    cpu = None
    roofline = None
    if not args.no_cpu:
        print("oracle on the host ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(pos, nc, grid, args.cpu_cubes,
                           other_grids=({"fp32_cell_local": cell_grid, "fp32_slab": slab_grid}
                                        if cell_grid is not None else None),
                           single_thread_cubes=10_000)
        pcnt = cpu.pop("_paper_counters")
        cnt = cpu.pop("_counters")
        nz_per_tet = cnt["n_nonzero"] / max(cnt["n_tet"], 1)
        own = own_work(pos, nc, args.model_cubes, 1024, nz_per_tet)
        own["gpu_events_per_tet"] = {k: v / ntet for k, v in gwork.items()}
        roofline = roofline_line("queue_kernel<float, 1024, 8, 8, false, 128, false>", kernel_ms, ntet, own,
                                 paper_ops_per_tet(pcnt), nz_per_tet * ntet,
                                 12.0 * p["np"] ** 3 + 4.0 * nc ** 3, peaks, clk.summary(),
                                 load_traffic("queue_kernel", WORKLOAD))

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "tets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": WORKLOAD,
            "particles": p["np"] ** 3,
            "tets": ntet,
            "grid": [nc, nc, nc],
            "rms_displacement_spacings": p["rms"],
            "seed": p["seed"],
            "path": "exact cumulative-fraction clipping in FP64, FP32 output grid, FP64 mass sum",
        },
        "mass_error": mass_err,
        "gpu_counters": gstats,
        "clock": clk.summary(),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "surrogate": sur,
        "peaks": peaks,
        "fp64_grid": {"tets_per_s": ntet / (ms64 / 1e3), "ms": ms64},
        "fp32_cell_local": ({"tets_per_s": ntet / (ms_cell / 1e3), "ms": ms_cell,
                             "block_l1": (cpu or {}).get("fp32_cell_local_block_l1")}
                            if ms_cell else None),
        "fp32_slab": ({"tets_per_s": ntet / (ms_slab / 1e3), "ms": ms_slab,
                       "block_l1": (cpu or {}).get("fp32_slab_block_l1"),
                       "speedup_vs_cell_local": ms_cell / ms_slab}
                      if ms_slab else None),
    }
    if cpu is not None and "gpu_block_l1" in cpu:
        line["density_l1_sampled_block"] = cpu["gpu_block_l1"]
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
