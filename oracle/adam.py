"""Adam with a linear learning-rate schedule, and the per-kernel optimisation
loop of Sec. 4.4 / Sec. 5.1 (FP64).

Test infrastructure only (see ``oracle/__init__``).

Readings:
* Adam as published by Kingma & Ba (bias-corrected first and second moments),
  beta = (0.9, 0.999), eps = 1e-8 unless given; one learning rate for offsets
  and weights.
* Linear decay: at step s = 0..S-1, lr_s = lr0 + (lr1 - lr0) * s / (S - 1)
  (constant when lr0 == lr1 or S == 1).
* The unit in which the learning rate moves tap offsets is unstated (Sec.
  5.1): pixels (offset_units = 0), or the target's half-width (M - 1) / 2
  (offset_units = 1), the unit of normalised sampling coordinates in which
  an M x M window spans [-1, 1]; the offsets' learning rate is then
  lr_s * (M - 1) / 2 pixels.  Weights always move at lr_s.
* The loop evaluates F_Theta(delta) before every update and stops as soon as
  the PSNR reaches the stop threshold, without updating; ``steps`` is the
  number of Adam updates applied.  After S updates the final Theta is
  evaluated once more.  Optimisation parity with the GPU is by loss/PSNR
  tolerance only: the iteration is non-convex and FP32 vs FP64 rounding
  separates trajectories (parity unpinned beyond that tolerance).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .adjoint import impulse_loss_grad
from . import loss as _loss


@dataclass
class OptParams:
    max_steps: int = 1000
    lr0: float = 1e-3
    lr1: float = 1e-4
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    psnr_stop_db: float = float("inf")
    loss: int = _loss.NMSE
    charb_eps: float = 1e-3
    offset_units: int = 0


def lr_at(s, S, lr0, lr1):
    if S <= 1:
        return float(lr0)
    return float(lr0 + (lr1 - lr0) * (s / (S - 1)))


def adam_update(theta, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t is 1-based).  ``lr`` is a scalar, or an array that
    broadcasts against theta (one rate per coordinate).  Returns new
    (theta, m, v)."""
    theta = np.asarray(theta, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def rate_units(side, offset_units):
    """Per-coordinate multiplier of the learning rate for (ox, oy, w)."""
    u = 0.5 * (side - 1) if offset_units == 1 else 1.0
    return np.array([u, u, 1.0])


def optimize(target, theta0, taps, p: OptParams, trace=None):
    """Fit Theta to a dense target by Adam on the impulse-response loss.
    Returns (theta, psnr_db, steps).  If ``trace`` is a list, the loss and
    PSNR before each update are appended to it."""
    theta = np.array(theta0, dtype=np.float64).reshape(-1, 3)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    unit = rate_units(np.asarray(target).shape[0], p.offset_units)
    for s in range(p.max_steps):
        loss, ps, g = impulse_loss_grad(target, theta, taps, p.loss, p.charb_eps)
        if trace is not None:
            trace.append((loss, ps))
        if ps >= p.psnr_stop_db:
            return theta, ps, s
        theta, m, v = adam_update(theta, g, m, v, s + 1, lr_at(s, p.max_steps, p.lr0, p.lr1) * unit,
                                  p.beta1, p.beta2, p.eps)
    loss, ps, _ = impulse_loss_grad(target, theta, taps, p.loss, p.charb_eps)
    if trace is not None:
        trace.append((loss, ps))
    return theta, ps, p.max_steps


def fit_continuation(targets, theta0, taps, scale, p: OptParams):
    """Basis precompute by continuation (the offline stage of Sec. 4.3, with
    the tap-correspondence reading: every entry shares one layer structure).
    Entry 0 starts from ``theta0``; entry k starts from the fitted entry k-1
    with its offsets multiplied by scale[k] and its weights kept.
    Returns (thetas [G][T][3], psnr_db [G], steps [G])."""
    thetas, psnrs, steps = [], [], []
    start = np.array(theta0, dtype=np.float64).reshape(-1, 3)
    for k, target in enumerate(targets):
        if k > 0:
            start = thetas[-1].copy()
            start[:, :2] *= scale[k]
        th, ps, st = optimize(target, start, taps, p)
        thetas.append(th)
        psnrs.append(ps)
        steps.append(st)
    return np.stack(thetas), np.array(psnrs), np.array(steps)
