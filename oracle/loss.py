"""Losses and fidelity metrics on the synthesised impulse response (FP64).

Test infrastructure only (see ``oracle/__init__``).

The paper trains with a Charbonnier loss between K_syn and K_tgt (Eq. 11) and
reports PSNR (Sec. 5.1, evaluation metrics) without stating the peak or the
Charbonnier epsilon.  Readings used here:
* MSE is normalised by the target's peak: NMSE = mean((K_syn - K_tgt)^2) /
  max(K_tgt)^2, so that Adam's epsilon does not swamp gradients of order
  1e-9 (kernels are normalised to unit sum).
* PSNR = 10 log10(max(K_tgt)^2 / MSE) = -10 log10(NMSE), over the M x M window.
* Charbonnier on the peak-normalised difference: mean(sqrt((d / peak)^2 + eps^2))
  with eps = 1e-3.
"""
from __future__ import annotations

import numpy as np

NMSE = 0
CHARBONNIER = 1


def peak(target):
    return float(np.max(np.asarray(target, dtype=np.float64)))


def nmse(ksyn, target):
    ksyn = np.asarray(ksyn, dtype=np.float64)
    target = np.asarray(target, dtype=np.float64)
    pk = peak(target)
    return float(np.mean((ksyn - target) ** 2) / (pk * pk))


def psnr_db(ksyn, target):
    e = nmse(ksyn, target)
    return float("inf") if e == 0.0 else float(-10.0 * np.log10(e))


def charbonnier(ksyn, target, eps=1e-3):
    """Eq. 11: the Charbonnier (smooth L1) penalty, mean over the window, on
    the peak-normalised difference."""
    d = (np.asarray(ksyn, np.float64) - np.asarray(target, np.float64)) / peak(target)
    return float(np.mean(np.sqrt(d * d + eps * eps)))


def loss_and_grad(ksyn, target, kind=NMSE, eps=1e-3):
    """(loss, dloss/dK_syn) for the chosen loss."""
    ksyn = np.asarray(ksyn, dtype=np.float64)
    target = np.asarray(target, dtype=np.float64)
    n = ksyn.size
    pk = peak(target)
    d = ksyn - target
    if kind == NMSE:
        return float(np.mean(d * d) / (pk * pk)), 2.0 * d / (n * pk * pk)
    if kind == CHARBONNIER:
        dn = d / pk
        s = np.sqrt(dn * dn + eps * eps)
        return float(np.mean(s)), dn / (s * n * pk)
    raise ValueError("unknown loss")
