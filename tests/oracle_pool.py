"""Process-parallel evaluation of the FP64 oracle for the large parity cases
(test infrastructure: imports only numpy and oracle/, never the GPU path).
Workers are spawned fresh processes, so they share nothing with a parent that
has a GPU context."""
from __future__ import annotations

import multiprocessing as mp
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np


def _one_step(job):
    from oracle import adam as Ad, adjoint as A
    K, th0, taps, lr, loss = job
    _, _, g = A.impulse_loss_grad(K.astype(np.float64), th0.astype(np.float64), taps, loss)
    th1, _, _ = Ad.adam_update(th0.astype(np.float64), g, np.zeros_like(g), np.zeros_like(g), 1, lr)
    return th1, g


def one_step_all(kernels, theta0s, taps, lr, loss=0, workers=None):
    """Oracle Theta after one Adam step, and the gradient, for every target.
    ``lr``: one rate for all, or a list with each target's rate (a scalar or
    one per coordinate)."""
    workers = workers or max(1, min(16, os.cpu_count() or 1))
    lrs = list(lr) if isinstance(lr, (list, tuple)) else [lr] * len(kernels)
    jobs = [(k, t, list(tp), r, loss) for k, t, tp, r in zip(kernels, theta0s, taps, lrs)]
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_one_step, jobs, chunksize=max(1, len(jobs) // (8 * workers))))


def _trajectory(job):
    from oracle import adam as Ad
    K, th0, taps, kw = job
    th, ps, st = Ad.optimize(K.astype(np.float64), th0.astype(np.float64), taps, Ad.OptParams(**kw))
    return th, ps, st


def trajectories(kernels, theta0s, taps, workers=None, **kw):
    """Oracle (Theta, PSNR, steps) after Ad.optimize with OptParams(**kw), per target."""
    workers = workers or max(1, min(16, os.cpu_count() or 1))
    jobs = [(k, t, list(tp), kw) for k, t, tp in zip(kernels, theta0s, taps)]
    with ProcessPoolExecutor(max_workers=min(workers, len(jobs)), mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_trajectory, jobs))
