"""Dense convolution (Eq. 1), uniform and spatially varying, in FP64: the
quality reference that the sparse chain approximates.

Test infrastructure only (see ``oracle/__init__``).

Orientation: out[p] = sum_q K[q] * I[clamp(p - q)] with q = (qx, qy) running
over the kernel's centred offsets and K[q] stored at row c + qy, column
c + qx.  This is the true convolution (the "*" of Eq. 3 / Eq. 4); Eq. 1 is
written as a correlation, which differs only by a 180-degree rotation of K.
The image boundary is clamp-to-edge, as for the sparse filter on images.
"""
from __future__ import annotations

import numpy as np


def _clamped(I, yy, xx):
    H, W = I.shape[-2:]
    return I[..., np.clip(yy, 0, H - 1), np.clip(xx, 0, W - 1)]


def dense_uniform(image, K, rows=None, cols=None):
    """Uniform dense convolution of image [C][H][W] (or [H][W]) with an odd
    square kernel K.  ``rows``/``cols`` (slices) restrict the output window;
    inputs are always read from the full image."""
    I = np.asarray(image, dtype=np.float64)
    K = np.asarray(K, dtype=np.float64)
    H, W = I.shape[-2:]
    rows = rows or slice(0, H)
    cols = cols or slice(0, W)
    y, x = np.mgrid[rows, cols]
    h = (K.shape[0] - 1) // 2
    out = np.zeros(I.shape[:-2] + y.shape)
    for qy in range(-h, h + 1):
        for qx in range(-h, h + 1):
            k = K[h + qy, h + qx]
            if k != 0.0:
                out += k * _clamped(I, y - qy, x - qx)
    return out


def dense_sv(image, coverage, pmap, half, rows=None, cols=None):
    """Spatially varying dense convolution: out[p] = sum_q K_{P(p)}[q] I[clamp(p-q)]
    with K_P[q] = coverage(P, q) / sum_q' coverage(P, q').

    ``coverage(P, qx, qy)`` returns the unnormalised weight of offset (qx, qy)
    for every parameter vector in P ([dims][h][w], the output window);
    ``half`` bounds the offsets, |qx|, |qy| <= half."""
    I = np.asarray(image, dtype=np.float64)
    P = np.asarray(pmap, dtype=np.float64)
    if P.ndim == 2:
        P = P[None]
    H, W = I.shape[-2:]
    rows = rows or slice(0, H)
    cols = cols or slice(0, W)
    y, x = np.mgrid[rows, cols]
    Pw = P[:, y, x]
    out = np.zeros(I.shape[:-2] + y.shape)
    Z = np.zeros(y.shape)
    for qy in range(-half, half + 1):
        for qx in range(-half, half + 1):
            k = coverage(Pw, qx, qy)
            Z += k
            out += k * _clamped(I, y - qy, x - qx)
    return out / Z


def disk_coverage(r_of_p):
    """Uniform disks of radius r(P[0]): coverage clamp(r + 1/2 - |q|, 0, 1)."""
    def coverage(P, qx, qy):
        return np.clip(r_of_p(P[0]) + 0.5 - np.hypot(qx, qy), 0.0, 1.0)
    return coverage


def ellipse_coverage(r_of_p, a_of_p):
    """Axis-aligned elliptical disks with semi-axes (r sqrt(a), r / sqrt(a)),
    r = r(P[0]), a = a(P[1]); coverage clamp(1/2 - d, 0, 1) with d the signed
    distance to the boundary measured along the ray from the centre."""
    def coverage(P, qx, qy):
        r = r_of_p(P[0])
        a = a_of_p(P[1])
        ax = r * np.sqrt(a)
        ay = r / np.sqrt(a)
        rho = np.hypot(qx / ax, qy / ay)
        nq = np.hypot(qx, qy)
        scale = np.where(rho > 0, nq / np.maximum(rho, 1e-300), np.minimum(ax, ay))
        return np.clip(0.5 - (rho - 1.0) * scale, 0.0, 1.0)
    return coverage
