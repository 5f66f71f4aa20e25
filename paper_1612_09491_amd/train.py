"""Train the learned overlap surrogate on the GPU.

Examples come from seeded Zel'dovich boxes that no evaluation uses (seeds from
synth.TRAIN_SEED0 up): 256^3 particles, rms displacement 2 spacings, deposited
onto a 64^3 grid (0.25 cells per Lagrangian spacing), where most tetrahedra
fit a 2x2x2 block of cells.  Labels are the exact overlap fractions from
psd_surrogate_examples; training runs the library's backward and Adam
kernels, batches drawn from a seeded permutation per epoch, with the learning
rate decaying geometrically over the run.

    python -m paper_1612_09491_amd.train --out surrogate.npy [--examples N] [--epochs E]

Writes the float32 parameters (numpy .npy) and a JSON record of the run next
to them.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import paper_1612_09491_amd as psd  # noqa: E402
from synth import TRAIN_SEED0, uniform_segments, zeldovich_positions  # noqa: E402

# fan-in of each parameter block (biases take their layer's)
_FAN_IN = {"W1": 12, "b1": 12, "W2": 64, "b2": 64, "W3": 64, "b3": 64, "W4": 64, "b4": 64}


def initial_parameters(seed: int) -> np.ndarray:
    """U(-1/sqrt(fan_in), 1/sqrt(fan_in)) per block, packed in the ABI's order."""
    segs = [(int(np.prod(shape)), 1.0 / math.sqrt(_FAN_IN[name]))
            for name, shape in psd.SURROGATE_LAYOUT]
    return uniform_segments(segs, seed)


def collect_examples(n_examples: int, np_: int = 256, rms: float = 2.0, nc: int = 64,
                     boxes: int = 4, seed0: int = TRAIN_SEED0, log=print) -> dict:
    """n_examples eligible tetrahedra (>= 2 cells) from `boxes` fresh-seed boxes, equal
    shares, each share from a contiguous run of Lagrangian cubes starting at cube 0."""
    dev = torch.device("cuda:0")
    per = (n_examples + boxes - 1) // boxes
    parts = []
    for b in range(boxes):
        want = min(per, n_examples - sum(len(p["mask"]) for p in parts))
        if want <= 0:
            break
        pos = torch.from_numpy(zeldovich_positions(np_, rms, seed0 + b)).to(dev)
        ex = psd.surrogate_examples(pos, nc, capacity=want, with_ids=False)
        if ex["found"] < want:
            raise RuntimeError(f"box {seed0 + b} holds only {ex['found']} examples")
        parts.append(ex)
        log(f"box seed {seed0 + b}: {want} examples")
        del pos
    return {k: torch.cat([p[k] for p in parts]) for k in ("feat", "frac", "mask")}


def train(params: torch.Tensor, ex: dict, epochs: int, batch: int, lr: float, lr_final: float,
          seed: int, log=print, steps_per_launch: int = 256) -> dict:
    n = int(ex["mask"].numel())
    rng = np.random.default_rng(seed)
    state = None
    steps_per_epoch = (n + batch - 1) // batch
    decay = (lr_final / lr) ** (1.0 / max(epochs * steps_per_epoch - 1, 1))
    history = []
    t0 = time.perf_counter()
    for e in range(epochs):
        order = rng.permutation(n).astype(np.int64)
        rate = lr * decay ** (e * steps_per_epoch)
        state = psd.train_surrogate(params, ex["feat"], ex["frac"], ex["mask"], order, batch=batch,
                                    lr=rate, lr_final=rate * decay ** (steps_per_epoch - 1),
                                    state=state, steps_per_launch=steps_per_launch)
        mean_loss = float(state["losses"].mean().item())
        history.append(mean_loss)
        log(f"epoch {e}: mean loss {mean_loss:.5f} ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    return {"epoch_loss": history, "seconds": time.perf_counter() - t0,
            "steps": int(state["step"]) if state else 0}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--examples", type=int, default=20_000_000)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--lr-final", type=float, default=2e-5)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--steps-per-launch", type=int, default=256,
                    help="Adam steps per cooperative launch (0: one backward and one Adam "
                         "launch per step)")
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    t0 = time.perf_counter()
    ex = collect_examples(args.examples, log=log)
    t_ex = time.perf_counter() - t0
    params = torch.from_numpy(initial_parameters(args.seed)).to("cuda:0")
    rec = train(params, ex, args.epochs, args.batch, args.lr, args.lr_final, args.seed + 1, log=log,
                steps_per_launch=args.steps_per_launch)
    w = params.cpu().numpy()
    np.save(args.out, w)
    rec.update({"examples": int(ex["mask"].numel()), "epochs": args.epochs, "batch": args.batch,
                "steps_per_launch": args.steps_per_launch,
                "lr": args.lr, "lr_final": args.lr_final, "init_seed": args.seed,
                "example_seconds": t_ex, "train_boxes": "zeldovich(256, rms 2.0) -> 64^3, "
                f"seeds {TRAIN_SEED0}..{TRAIN_SEED0 + 3}"})
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(rec, f, indent=1)
    log(json.dumps({k: v for k, v in rec.items() if k != "epoch_loss"}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
