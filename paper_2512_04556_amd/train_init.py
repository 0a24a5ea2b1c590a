"""Train the learned initialiser and write its parameters.

    python -m paper_2512_04556_amd.train_init [--n 150000] [--epochs 60] [--out PATH]

Training data: ``n`` synthetic targets (odd sides 15..127, the shape
families of the batched-optimisation workload, 4 layers x 12 taps), each
fitted by the batched optimiser from the radial initialisation (Adam, 1000
steps or 40 dB, lr 1e-2 -> 1e-3 with the offsets' rate in units of the
target's half-width, normalised MSE).  The network regresses the
fitted Theta in its own units (offsets / hw) from the area-resampled 64 x 64
input.  Everything on the GPU runs through libdisk; this script only moves
tensors around.  Chunk i of 4096 targets is drawn with seed 6000 + i.
"""
from __future__ import annotations

import argparse
import json
import os
import time
from multiprocessing import Pool

import numpy as np
import torch

from . import (OFFSETS_HALF_WIDTH, OptParams, disk_init_radial, disk_net_param_count, disk_net_prepare_inputs, disk_net_train_step,
               disk_optimize_batch, make_batch, net_workspace)

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "init_net.f32")
CHUNK = 4096
SHAPES = (64, 64)


def _chunk(args):
    i, n = args
    from synth import mixed_batch, pack_targets
    b = mixed_batch(n, seed=6000 + i, fixed_L=4, fixed_N=12)
    return pack_targets(b)


# the optimiser settings of the batched workloads (and of the comparison the
# network is judged by)
FIT = dict(lr0=1e-2, lr1=1e-3, psnr_stop_db=40.0, offset_units=OFFSETS_HALF_WIDTH)


def fitted_pairs(n, steps=1000, workers=8, log=print):
    """(inputs int16 [n][64][64] BF16 bits, half_width [n], theta [n][48][3],
    psnr [n]) on the GPU."""
    sizes = [min(CHUNK, n - o) for o in range(0, n, CHUNK)]
    with Pool(workers) as pool:
        packed = pool.map(_chunk, list(enumerate(sizes)))
    xs, hws, ths, pss = [], [], [], []
    prm = OptParams(max_steps=steps, **FIT)
    for i, (desc, taps, tg) in enumerate(packed):
        t = time.perf_counter()
        bt = make_batch(desc, taps, tg)
        th = disk_init_radial(bt)
        ps, st, _ = disk_optimize_batch(bt, th, prm)
        x, hw = disk_net_prepare_inputs(bt)
        torch.cuda.synchronize()
        xs.append(x)
        hws.append(hw)
        ths.append(th.view(-1, 48, 3))
        pss.append(ps)
        log(f"chunk {i}: {bt.B} targets fitted in {time.perf_counter() - t:.2f} s, "
            f"median PSNR {float(ps.median()):.1f} dB, median steps {float(st.float().median()):.0f}")
    return torch.cat(xs), torch.cat(hws), torch.cat(ths), torch.cat(pss)


def init_params(seed=0):
    """Kaiming-uniform weights (bound sqrt(6 / fan_in)), zero biases, in the
    blob order of libdisk (PyTorch layout per layer)."""
    g = np.random.default_rng(seed)
    widths = [1, 32, 64, 128, 128, 256, 256]
    parts = []
    for i in range(6):
        fan_in = widths[i] * 9
        parts.append(g.uniform(-1, 1, widths[i + 1] * fan_in) * np.sqrt(6.0 / fan_in))
        parts.append(np.zeros(widths[i + 1]))
    for fin, fout in ((256, 512), (512, 144)):
        parts.append(g.uniform(-1, 1, fin * fout) * np.sqrt(6.0 / fin))
        parts.append(np.zeros(fout))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == disk_net_param_count()
    return torch.as_tensor(p).cuda()


def train(x, hw, theta, epochs=40, batch=256, lr=1e-3, val=2048, seed=0, log=print):
    n = x.shape[0]
    gen = torch.Generator().manual_seed(seed)
    perm = torch.randperm(n, generator=gen).cuda()
    vi, ti = perm[:val], perm[val:]
    params = init_params(seed)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    ws = net_workspace(batch)
    vws = net_workspace(val)
    step = 0
    total = epochs * (ti.numel() // batch)
    hist = []
    for ep in range(epochs):
        t = time.perf_counter()
        order = ti[torch.randperm(ti.numel(), generator=gen).cuda()]
        losses = []
        for k in range(ti.numel() // batch):
            idx = order[k * batch:(k + 1) * batch]
            step += 1
            lr_t = lr * 0.5 * (1.0 + np.cos(np.pi * (step - 1) / total))   # cosine decay
            losses.append(disk_net_train_step(params, m, v, step, lr_t, x[idx].contiguous(), hw[idx].contiguous(),
                                              theta[idx].contiguous(), ws=ws))
        # validation loss: a step with lr 0 on scratch copies leaves params unchanged
        vl = disk_net_train_step(params.clone(), torch.zeros_like(params), torch.zeros_like(params), 1, 0.0,
                                 x[vi].contiguous(), hw[vi].contiguous(), theta[vi].contiguous(), ws=vws)
        torch.cuda.synchronize()
        tl = float(torch.stack(losses).mean())
        hist.append((ep, tl, float(vl)))
        log(f"epoch {ep}: train {tl:.5f} val {float(vl):.5f} ({time.perf_counter() - t:.2f} s)")
    return params, hist


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=150000)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--out", default=WEIGHTS)
    a = ap.parse_args()
    t0 = time.perf_counter()
    x, hw, theta, ps = fitted_pairs(a.n, a.steps, log=lambda s: print(s, flush=True))
    t1 = time.perf_counter()
    params, hist = train(x, hw, theta, epochs=a.epochs, log=lambda s: print(s, flush=True))
    t2 = time.perf_counter()
    params.cpu().numpy().astype("<f4").tofile(a.out)
    meta = {"n": a.n, "epochs": a.epochs, "steps": a.steps, "fit": {k: v for k, v in FIT.items()},
            "data_seconds": round(t1 - t0, 1),
            "train_seconds": round(t2 - t1, 1), "final": hist[-1], "median_psnr_db": float(ps.median())}
    with open(a.out + ".json", "w") as f:
        json.dump(meta, f, indent=1)
    print(json.dumps(meta), flush=True)


def load(path=WEIGHTS, device="cuda"):
    """The trained parameters as a device tensor (raises if missing)."""
    p = np.fromfile(path, dtype="<f4")
    if p.size != disk_net_param_count():
        raise ValueError(f"{path}: {p.size} values, expected {disk_net_param_count()}")
    return torch.as_tensor(p).to(device)


if __name__ == "__main__":
    main()
