"""Helpers shared by the GPU parity tests (no method arithmetic here)."""
import sys

import numpy as np
import torch


def say(*a):
    """Name the case before a GPU step, flushed, so a failing run shows it."""
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def to_dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def to_np(t):
    torch.cuda.synchronize()
    return t.detach().float().cpu().numpy().astype(np.float64)


def bf16_round(a):
    """float32 -> bfloat16 -> float64 (round to nearest even), on the CPU."""
    return torch.as_tensor(np.asarray(a, np.float32)).bfloat16().float().numpy().astype(np.float64)


def rel_err(got, want):
    """max |got - want| / max |want| (the error figure quoted in every test)."""
    want = np.asarray(want, np.float64)
    pk = float(np.abs(want).max())
    return float(np.abs(np.asarray(got, np.float64) - want).max()) / (pk if pk > 0 else 1.0)


TOL_F32 = 1e-5     # max-abs error relative to the peak, FP32 path
TOL_BF16 = 5e-3    # the same with BF16 image I/O
