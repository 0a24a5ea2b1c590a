"""Spatially varying sparse filtering (Sec. 4.3) in FP64.

Test infrastructure only (see ``oracle/__init__``).

At every pixel the parameter map P selects interpolation weights over the
basis (``oracle.interp``), the per-pixel Theta(x, y) is the convex combination
of the basis entries (Eq. 9), and the L sparse layers are applied as in the
uniform chain with that pixel's taps:
    X_l[p] = sum_i w_{l,i}(p) * B_CLAMP(X_{l-1}, p - o_{l,i}(p)).
Readings: the filter is a gather (each output pixel uses its own filter), the
same per-pixel Theta serves every pass, the canvas is the image with a CLAMP
boundary at every pass.
"""
from __future__ import annotations

import numpy as np

from .sparse import CLAMP, bilinear_offset, pixel_grid
from .interp import tap_field


def sv_chain(image, pmap, basis, grid, taps, keep=False):
    """image: [C][H][W]; pmap: [dims][H][W] with dims = len(grid);
    basis: [prod(grid)][T][3].  Returns X_L [C][H][W] (or all X_l)."""
    X = np.asarray(image, dtype=np.float64)
    P = np.asarray(pmap, dtype=np.float64)
    if P.ndim == 2:
        P = P[None]
    H, W = X.shape[-2:]
    px, py = pixel_grid(H, W)
    Xs = [X]
    t0 = 0
    for N in taps:
        Y = np.zeros_like(Xs[-1])
        for i in range(t0, t0 + int(N)):
            ox, oy, w = tap_field(basis, P, grid, i)
            Y += w * bilinear_offset(Xs[-1], px, py, ox, oy, CLAMP)
        t0 += int(N)
        Xs.append(Y)
    return Xs if keep else Xs[-1]
