"""Autotuner of the persistent optimiser's launch shape.

    python -m paper_2512_04556_amd.autotune [--out PATH] [--steps N] [--reps R]

For each cell of (batch size, largest side, largest tap count) it builds a
seeded batch (odd sides uniform over 15 .. the cell's side, the shape families of
the batched workload, radial initialisation; 4 layers x 12 taps for the cells
of up to 48 taps, else 2..6 layers of 6..16 taps), times every candidate
shape (256-thread work-groups with 1..4 resident per compute unit, 1024-thread
work-groups with one per unit) on up to N Adam steps under the batched
workload's settings (learning rates, offset units, stopping at 40 dB, so that
targets leave the queue when they converge and the largest ones set the
end, as in real batches), and
keeps the fastest.  The table it writes (the C rows of opt_tune_table.inc) is
what disk_optimize_batch uses when called without a tune argument; a summary
of every timing goes to stdout as JSON lines.
"""
from __future__ import annotations

import argparse
import json
import os

import torch

from . import OptParams, disk_init_radial, disk_optimize_batch, make_batch, opt_tune, optimize_workspace_size

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "csrc", "opt_tune_table.inc")
CANDIDATES = [(256, 1), (256, 2), (256, 3), (256, 4), (1024, 1)]
# measured batch sizes and the largest batch each row then covers
BATCHES = [(1, 4), (16, 32), (64, 128), (256, 512), (1024, 2048), (4096, 1 << 30)]
# side ranges of the cells: a batch whose largest side is hi usually holds
# smaller targets too, so each cell draws from 15 .. hi (the largest target
# then sets the critical path as it would in such a batch)
SIDES = [(15, 31), (15, 63), (15, 127), (15, 255)]
# largest tap count a row covers, and the layer / tap mix of its batches
TAPS = [(48, {"fixed_L": 4, "fixed_N": 12}), (1 << 30, {})]


def time_shape(bt, th0, prm, shape, reps=2):
    ws = torch.empty(optimize_workspace_size(bt, opt_tune(shape[1], shape[0])), dtype=torch.uint8, device="cuda")
    best = float("inf")
    for _ in range(reps + 1):                 # the first run warms up
        th = th0.clone()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        disk_optimize_batch(bt, th, prm, tune=opt_tune(shape[1], shape[0]), ws=ws)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def main():
    from synth import mixed_batch, pack_targets
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--reps", type=int, default=1)
    a = ap.parse_args()
    from .train_init import FIT
    prm = OptParams(max_steps=a.steps, **FIT)
    rows = []
    for B, max_B in BATCHES:
        for lo, hi in SIDES:
            for max_T, mix in TAPS:
                b = mixed_batch(B, seed=9000 + B + hi, side=(lo, hi), **mix)
                bt = make_batch(*pack_targets(b))
                th0 = disk_init_radial(bt)
                times = {f"{t}x{w}": round(time_shape(bt, th0, prm, (t, w), a.reps), 4) for t, w in CANDIDATES}
                best = min(CANDIDATES, key=lambda c: times[f"{c[0]}x{c[1]}"])
                rows.append((max_B, hi, max_T, best[0], best[1]))
                print(json.dumps({"B": B, "sides": [lo, hi], "max_T": bt.meta.max_T, "steps": a.steps, "ms": times,
                                  "best": list(best)}), flush=True)
    with open(a.out, "w") as f:
        f.write("// written by paper_2512_04556_amd/autotune.py; do not edit by hand\n")
        f.write("// rows: {max_B, max_side_upto, max_T_upto, threads, wgs_per_cu}, first match wins\n")
        f.write("static const TuneRow kTuneRows[] = {\n")
        for r in rows:
            f.write(f"    {{{r[0]}, {r[1]}, {r[2]}, {r[3]}, {r[4]}}},\n")
        f.write("};\n")


if __name__ == "__main__":
    main()
