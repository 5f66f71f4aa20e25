"""Benchmark: tetrahedra deposited per second on one MI355X.

Workload: 256^3 particles on a periodic unit box (Zel'dovich displacement,
rms 2 spacings, seed 2) -> 100,663,296 tetrahedra deposited exactly onto a
512^3 FP32 grid.  One step = one full psd_deposit_uniform call (output
zeroing, tetrahedron generation, cell walk, exact clipping in FP64, scatter,
FP64 mass sum) with the positions already resident in HBM.

Prints ONE JSON line.  Also reports:
  roofline      the deposit kernel's algorithmic lane-operations per second
                against the chip's VALU issue rate (the path is ALU-bound);
  cpu_baseline  the FP64 oracle timed on a seeded sample of the same
                workload on the host cores, with its sampled-block density
                error of the GPU result;
  surrogate     the learned-surrogate path (trained weights from
                paper_1612_09491_amd/train.py) in tets/s with its whole-grid
                density L1 against the exact GPU grid, on this workload and on
                256^3 -> 64^3, where most tetrahedra are eligible.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "tetrahedra deposited/sec on 1 MI355X, exact vs surrogate at stated density L1 error"
WORKLOAD = "zel256_g512"

# VALU issue rate: 256 CUs x 64 lanes x 2.4 GHz (one lane-op per lane per clock).
SIMDS = 256 * 4            # compute units x SIMDs, MI355X
CLOCK_HZ = 2.4e9           # peak engine clock
PEAK_VALU_OPS = 256 * 64 * CLOCK_HZ

# Unit costs (lane-ops) of the paper's method, per counted event: tetrahedron
# setup, bbox-cell classification, signed distance per vertex per plane visit,
# edge cut, sub-tetrahedron volume, scatter of a non-zero deposit.
COST = {"tet": 60, "pair": 24, "pv": 4, "cut": 9, "sub": 20, "nz": 2}


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


def algorithmic_ops_per_tet(cnt: dict) -> float:
    n = max(cnt["n_tet"], 1)
    return (COST["tet"] * cnt["n_tet"] + COST["pair"] * cnt["n_pair"] + COST["pv"] * cnt["n_pv"] +
            COST["cut"] * cnt["n_cut"] + COST["sub"] * cnt["n_sub"] +
            COST["nz"] * cnt["n_nonzero"]) / n


def cpu_baseline(pos: np.ndarray, nc: int, gpu_grid: np.ndarray | None, n_cubes: int,
                 seed: int = 12345, other_grids: dict | None = None) -> dict:
    """The FP64 oracle on a seeded random sample of Lagrangian cubes, on host cores."""
    import oracle
    oracle.build_oracle(force=False)
    npart = pos.shape[0]
    rng = np.random.default_rng(seed)
    cubes = np.sort(rng.choice(npart ** 3, size=n_cubes, replace=False)).astype(np.int64)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
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
                  f"seed {seed}, FP64 polytope clipper, {dt:.1f} s",
        "counters_per_tet": {k: v / max(pcnt["n_tet"], 1) for k, v in pcnt.items()},
    }
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
    return out


# template arguments after the buffer size of each deposit-kernel instance:
# tets set up at once, tiles per batch
GROUP_OF_CAP = {512: "16, 16", 960: "32, 16", 1408: "8, 8", 2048: "32, 32"}

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


def surrogate_leg(psd, torch, pt, p, exact_grid, reps: int) -> dict | None:
    """The surrogate path beside the exact one: tets/s and whole-grid density L1 against
    the exact GPU grid, on the benchmark workload and on the 0.25-cells-per-spacing one."""
    if not os.path.exists(SURROGATE_WEIGHTS):
        return None
    from synth import workload
    w = torch.from_numpy(np.load(SURROGATE_WEIGHTS).astype(np.float32)).to(pt.device)
    ntet = 6 * p["np"] ** 3
    st = torch.zeros(8, dtype=torch.int64, device=pt.device)
    ms, grid = time_deposit(psd, torch, pt, p["nc"], psd.PSD_SURROGATE, reps, surrogate=w)
    psd.deposit_uniform(pt, p["nc"], flags=psd.PSD_SURROGATE, stats=st, surrogate=w)
    out = {"weights": os.path.basename(SURROGATE_WEIGHTS),
           WORKLOAD: {"tets_per_s": ntet / (ms / 1e3), "ms": ms,
                      "eligible_tets": int(st[6].item()),
                      "density_l1_vs_exact": rel_l1(grid.double(), exact_grid)}}
    pos2, p2 = workload("zel256_g64")
    pt2 = torch.from_numpy(pos2).to(pt.device)
    ntet2 = 6 * p2["np"] ** 3
    ms_x, g_x = time_deposit(psd, torch, pt2, p2["nc"], 0, reps)
    ms_s, g_s = time_deposit(psd, torch, pt2, p2["nc"], psd.PSD_SURROGATE, reps, surrogate=w)
    st.zero_()
    psd.deposit_uniform(pt2, p2["nc"], flags=psd.PSD_SURROGATE, stats=st, surrogate=w)
    out["zel256_g64"] = {"exact_tets_per_s": ntet2 / (ms_x / 1e3),
                         "surrogate_tets_per_s": ntet2 / (ms_s / 1e3),
                         "eligible_tets": int(st[6].item()), "tets": ntet2,
                         "density_l1_vs_exact": rel_l1(g_s.double(), g_x.double())}
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
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    rng = np.random.default_rng(seed)
    total = sum(b.shape[0] * b.shape[1] * b.shape[2] for b in boxes)
    dt, tets = 0.0, 0
    pc = None
    for i, pos in enumerate(boxes):
        nb = pos.shape[0] * pos.shape[1] * pos.shape[2]
        k = max(16, int(round(n_cubes_total * nb / total)))
        k = min(k, nb)
        cubes = np.sort(rng.choice(nb, size=k, replace=False)).astype(np.int64)
        t0 = time.perf_counter()
        oracle.deposit_uniform(pos, nc_of(i), cubes=cubes, mode=oracle.TRIVIAL, nthreads=threads)
        dt += time.perf_counter() - t0
        tets += 6 * k
        _, c = oracle.deposit_uniform(pos, nc_of(i), cubes=cubes,
                                      mode=oracle.TRIVIAL | oracle.PAPER, nthreads=threads)
        # weight each box's counters by its share of all tetrahedra
        w = nb / total / (6 * k)
        pc = {key: (pc[key] if pc else 0.0) + v * w for key, v in c.items()}
    return {"seconds": dt, "tets": tets, "threads": threads, "ops_per_tet":
            algorithmic_ops_per_tet({k: v for k, v in pc.items()} | {"n_tet": 1.0})}


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
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1e3 / args.steps
    kernel_ms = e0.elapsed_time(e1) / args.steps
    finest = int(np.nonzero(levels)[0].max())
    nc_f = p["block"] << finest
    line = {"value": ntet / (ms_per_step / 1e3), "ms_per_step": ms_per_step,
            "dtype": "f64",
            "config": {"workload": "clump512_octree", "particles": p["np"] ** 3, "tets": ntet,
                       "leaves": tree.n_leaves, "nodes": tree.n_nodes,
                       "leaves_per_level": levels.tolist(), "block": p["block"],
                       "threshold": p["threshold"], "build_octree_ms": build_ms,
                       "path": "exact cumulative clipping in FP64 into 16^3 FP32 density leaves"},
            "mass_error": abs(float(ms.item()) - 1.0)}
    if not args.no_cpu:
        # the finest level's cells as a uniform grid carry the same algorithmic work
        o = oracle_sample_counts([pos], args.cpu_cubes, 12345, lambda i: nc_f)
        line["cpu_baseline"] = {"value": o["tets"] / o["seconds"], "unit": "tets/s",
                                "cores": o["threads"], "kind": "oracle",
                                "sample": f"{o['tets'] // 6} random Lagrangian cubes deposited "
                                          f"onto the finest level's {nc_f}^3 cells, "
                                          f"{o['seconds']:.1f} s"}
        achieved = o["ops_per_tet"] * ntet / (kernel_ms / 1e3)
        line["roofline"] = {"bound": "alu", "achieved": achieved / 1e12,
                            "peak": PEAK_VALU_OPS / 1e12, "unit": "Top/s",
                            "frac": achieved / PEAK_VALU_OPS, "traffic": None,
                            "kernel": "queue_kernel<float, 960, 32, 16>", "kernel_ms": kernel_ms,
                            "algorithmic_ops_per_tet": o["ops_per_tet"]}
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
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1e3 / args.steps
    kernel_ms = e0.elapsed_time(e1) / args.steps
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
                                "cores": o["threads"], "kind": "oracle",
                                "sample": f"{o['tets'] // 6} random Lagrangian cubes spread over "
                                          f"the 64 boxes by size, {o['seconds']:.1f} s"}
        achieved = o["ops_per_tet"] * ntet / (kernel_ms / 1e3)
        line["roofline"] = {"bound": "alu", "achieved": achieved / 1e12,
                            "peak": PEAK_VALU_OPS / 1e12, "unit": "Top/s",
                            "frac": achieved / PEAK_VALU_OPS, "traffic": None,
                            "kernel": f"queue_kernel<float, {best[0]}, {GROUP_OF_CAP[best[0]]}>", "kernel_ms": kernel_ms,
                            "algorithmic_ops_per_tet": o["ops_per_tet"]}
    return line


def bench_surrogate_workload(args, torch, psd) -> dict:
    """256^3 -> 64^3 (0.25 cells per spacing, ~72% of tets eligible for the network):
    the exact path and the surrogate path on the same positions."""
    from synth import workload
    dev = torch.device("cuda:0")
    pos, p = workload("zel256_g64")
    nc = p["nc"]
    ntet = 6 * p["np"] ** 3
    pt = torch.from_numpy(pos).to(dev)
    if not os.path.exists(SURROGATE_WEIGHTS):
        raise SystemExit(f"{SURROGATE_WEIGHTS} is missing: train with paper_1612_09491_amd/train.py")
    w = torch.from_numpy(np.load(SURROGATE_WEIGHTS).astype(np.float32)).to(dev)
    reps = max(1, args.steps)
    ms_x, g_x = time_deposit(psd, torch, pt, nc, 0, reps)
    ms_s, g_s = time_deposit(psd, torch, pt, nc, psd.PSD_SURROGATE, reps, surrogate=w)
    st = torch.zeros(8, dtype=torch.int64, device=dev)
    psd.deposit_uniform(pt, nc, flags=psd.PSD_SURROGATE, stats=st, surrogate=w)
    line = {"value": ntet / (ms_s / 1e3), "ms_per_step": ms_s, "dtype": "bf16+f64",
            "config": {"workload": "zel256_g64", "particles": p["np"] ** 3, "tets": ntet,
                       "grid": [nc, nc, nc], "rms_displacement_spacings": p["rms"],
                       "seed": p["seed"], "weights": os.path.basename(SURROGATE_WEIGHTS),
                       "path": "learned surrogate (BF16 MFMA) for tets within 2x2x2 cells, "
                               "exact FP64 for the others"},
            "eligible_tets": int(st[6].item()),
            "density_l1_vs_exact": rel_l1(g_s.double(), g_x.double()),
            "exact": {"tets_per_s": ntet / (ms_x / 1e3), "ms": ms_x}}
    if not args.no_cpu:
        o = oracle_sample_counts([pos], args.cpu_cubes, 12345, lambda i: nc)
        line["cpu_baseline"] = {"value": o["tets"] / o["seconds"], "unit": "tets/s",
                                "cores": o["threads"], "kind": "oracle",
                                "sample": f"{o['tets'] // 6} random Lagrangian cubes, exact FP64 "
                                          f"polytope clipper, {o['seconds']:.1f} s"}
    return line


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-cubes", type=int, default=None,
                    help="Lagrangian cubes in the oracle's timed sample (default per workload, "
                         "about 10-30 s of host work)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate leg")
    ap.add_argument("--no-cell", action="store_true",
                    help="skip the per-cell (cell-local FP32) method's timing")
    ap.add_argument("--workload", default=WORKLOAD,
                    choices=[WORKLOAD, "clump512_octree", "batched64", "zel256_g64"],
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
              "zel256_g64": bench_surrogate_workload}[args.workload]
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
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = ntet / (ms_per_step / 1e3)
    mass_err = abs(float(msum.item()) - 1.0)
    grid = out.double().cpu().numpy()

    # Dominant kernel alone: accumulate mode skips the grid fill, so events on
    # the launch stream bracket the deposit kernel plus a one-wave counter reset.
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    kreps = max(1, min(args.steps, 3))
    scratch = torch.zeros_like(out)
    e0.record(stream)
    for _ in range(kreps):
        psd.deposit_uniform(pt, nc, out=scratch, flags=psd.PSD_ACCUMULATE, workspace=ws,
                            stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    kernel_ms = e0.elapsed_time(e1) / kreps
    st = torch.zeros(8, dtype=torch.int64, device=dev)
    psd.deposit_uniform(pt, nc, out=scratch, stats=st, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    gstats = dict(zip(psd.STAT_NAMES, (int(x) for x in st.cpu().numpy()[:6])))
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # the same deposit into an FP64 grid (identical arithmetic, double atomics)
    ms64, _ = time_deposit(psd, torch, pt, nc, psd.PSD_PREC_FP64, reps=max(1, min(args.steps, 2)))
    # the per-cell method: cell-local FP32 clipping (one timed run)
    ms_cell, cell_grid = (None, None)
    if not args.no_cell:
        ms_cell, g = time_deposit(psd, torch, pt, nc, psd.PSD_METHOD_CELL, reps=1)
        cell_grid = g.double().cpu().numpy()
        del g

    sur = None
    if not args.no_surrogate:
        sur = surrogate_leg(psd, torch, pt, p, out.double(), reps=max(1, min(args.steps, 3)))

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(pos, nc, grid, args.cpu_cubes,
                           other_grids={"fp32_cell_local": cell_grid} if cell_grid is not None else None)

    roofline = None
    if cpu is not None:
        ops_per_tet = algorithmic_ops_per_tet(cpu.pop("_paper_counters"))
        ops = ops_per_tet * ntet
        achieved = ops / (kernel_ms / 1e3)
        traffic = load_traffic("queue_kernel", WORKLOAD)
        roofline = {
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": PEAK_VALU_OPS / 1e12,
            "unit": "Top/s",
            "frac": achieved / PEAK_VALU_OPS,
            "traffic": traffic["bytes_per_launch"] if traffic else None,
            "kernel": "queue_kernel<float, 1408, 8, 8>",
            "kernel_ms": kernel_ms,
            "algorithmic_ops_per_tet": ops_per_tet,
        }
        if traffic and traffic.get("valu_insts_per_launch"):
            # machine view of the same launch: wave64 VALU instructions (rocprofv3
            # SQ_INSTS_VALU of this kernel version) x 4 clocks over 1024 SIMDs
            roofline["valu_issue_frac"] = (4.0 * traffic["valu_insts_per_launch"] /
                                           (SIMDS * CLOCK_HZ * kernel_ms / 1e3))

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
        "roofline": roofline,
        "cpu_baseline": cpu,
        "surrogate": sur,
        "fp64_grid": {"tets_per_s": ntet / (ms64 / 1e3), "ms": ms64},
        "fp32_cell_local": ({"tets_per_s": ntet / (ms_cell / 1e3), "ms": ms_cell,
                             "block_l1": (cpu or {}).get("fp32_cell_local_block_l1")}
                            if ms_cell else None),
    }
    if cpu is not None and "gpu_block_l1" in cpu:
        line["density_l1_sampled_block"] = cpu["gpu_block_l1"]
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
