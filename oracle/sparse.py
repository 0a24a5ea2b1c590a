"""Sparse layers, the nested chain and its impulse response (FP64).

Test infrastructure only (see ``oracle/__init__``).

Conventions (readings of the paper, all stated in the design notes):
* An image is ``X[..., H, W]`` (leading channel axes allowed), row = y,
  column = x, pixel centres at integer coordinates.
* A sparse kernel is a set of (offset o in R^2, weight w) pairs (Sec. 3.2,
  Eq. 2).  The paper does not name the sub-pixel rule for continuous offsets;
  this oracle uses bilinear interpolation, the minimal differentiable rule.
* A layer gathers at ``p - o``: Y[p] = sum_i w_i * B(X, p - o_i).  A tap's
  weight then lands at ``c + o_i`` in the impulse response, and filtering an
  image is the true convolution with the synthesised kernel (the "*" of Eq. 3
  and Eq. 4 and the LSI characterisation of Sec. 4.4).
* Boundary: ZERO (reads outside the canvas give 0) for the impulse canvas,
  CLAMP (indices clamped to the edge, weights unchanged) for images.
* Theta is a float [T][3] array of rows (ox, oy, w), layer-major, with
  ``taps[l]`` rows for layer l (the parameter set of Eq. 5).
"""
from __future__ import annotations

import numpy as np

ZERO = 0
CLAMP = 1


def split_layers(theta, taps):
    """Split layer-major [T][3] parameters into a list of per-layer [N_l][3]
    float64 arrays (Eq. 5: Theta is the union over layers)."""
    theta = np.asarray(theta, dtype=np.float64).reshape(-1, 3)
    taps = [int(t) for t in taps]
    if sum(taps) != theta.shape[0]:
        raise ValueError("sum(taps) != rows of theta")
    out, o = [], 0
    for n in taps:
        out.append(theta[o:o + n])
        o += n
    return out


def _read(X, yy, xx, boundary):
    """X[..., yy, xx] with the boundary rule applied to integer index arrays."""
    H, W = X.shape[-2:]
    if boundary == CLAMP:
        return X[..., np.clip(yy, 0, H - 1), np.clip(xx, 0, W - 1)]
    if boundary == ZERO:
        inside = (yy >= 0) & (yy < H) & (xx >= 0) & (xx < W)
        v = X[..., np.clip(yy, 0, H - 1), np.clip(xx, 0, W - 1)]
        return np.where(inside, v, 0.0)
    raise ValueError("boundary must be ZERO or CLAMP")


def bilinear(X, sx, sy, boundary):
    """B(X, s): bilinear read of X at continuous positions s = (sx, sy).

    x0 = floor(sx), fx = sx - x0 (same for y); the four neighbours are weighted
    (1-fx)(1-fy), fx(1-fy), (1-fx)fy, fx fy.  ``sx``/``sy`` are arrays of the
    output's spatial shape; X may carry leading channel axes.
    """
    X = np.asarray(X, dtype=np.float64)
    sx = np.asarray(sx, dtype=np.float64)
    sy = np.asarray(sy, dtype=np.float64)
    x0 = np.floor(sx)
    y0 = np.floor(sy)
    fx = sx - x0
    fy = sy - y0
    x0 = x0.astype(np.int64)
    y0 = y0.astype(np.int64)
    return ((1.0 - fx) * (1.0 - fy) * _read(X, y0, x0, boundary)
            + fx * (1.0 - fy) * _read(X, y0, x0 + 1, boundary)
            + (1.0 - fx) * fy * _read(X, y0 + 1, x0, boundary)
            + fx * fy * _read(X, y0 + 1, x0 + 1, boundary))


def bilinear_offset(X, px, py, ox, oy, boundary):
    """B(X, p - o) for integer pixel coordinates p and offsets o.

    Identical to ``bilinear(X, px - ox, py - oy)`` in exact arithmetic; the
    integer part is formed as p + floor(-o) and the fraction as
    -o - floor(-o), so no rounding of p - o can move a sample across an
    integer (where the read's derivative is discontinuous) when |o| is below
    the spacing of floats near p."""
    X = np.asarray(X, dtype=np.float64)
    nox = -np.asarray(ox, dtype=np.float64)
    noy = -np.asarray(oy, dtype=np.float64)
    fl_x = np.floor(nox)
    fl_y = np.floor(noy)
    fx = nox - fl_x
    fy = noy - fl_y
    x0 = (np.asarray(px) + fl_x).astype(np.int64)
    y0 = (np.asarray(py) + fl_y).astype(np.int64)
    return ((1.0 - fx) * (1.0 - fy) * _read(X, y0, x0, boundary)
            + fx * (1.0 - fy) * _read(X, y0, x0 + 1, boundary)
            + (1.0 - fx) * fy * _read(X, y0 + 1, x0, boundary)
            + fx * fy * _read(X, y0 + 1, x0 + 1, boundary))


def pixel_grid(H, W):
    """Integer pixel-centre coordinates (x, y), each of shape [H][W]."""
    y, x = np.mgrid[0:H, 0:W]
    return x.astype(np.float64), y.astype(np.float64)


def sparse_layer(X, layer, boundary):
    """One sparse layer (Eq. 2 applied as a convolution step of Eq. 3):
    Y[p] = sum_i w_i * B(X, p - o_i), for a spatially uniform [N][3] layer."""
    X = np.asarray(X, dtype=np.float64)
    H, W = X.shape[-2:]
    px, py = pixel_grid(H, W)
    Y = np.zeros_like(X)
    for ox, oy, w in np.asarray(layer, dtype=np.float64):
        Y += w * bilinear_offset(X, px, py, ox, oy, boundary)
    return Y


def chain(X, theta, taps, boundary, keep=False):
    """The nested convolution of Eq. 3: X_l = layer_l(X_{l-1}), l = 1..L, on
    a fixed canvas with one boundary rule.  Returns X_L, or the list
    [X_0, X_1, ..., X_L] when ``keep``."""
    Xs = [np.asarray(X, dtype=np.float64)]
    for layer in split_layers(theta, taps):
        Xs.append(sparse_layer(Xs[-1], layer, boundary))
    return Xs if keep else Xs[-1]


def impulse(H, W=None):
    """The discrete Dirac delta of Eq. 10: one non-zero pixel at the centre
    c = ((W-1)//2, (H-1)//2)."""
    W = H if W is None else W
    d = np.zeros((H, W))
    d[(H - 1) // 2, (W - 1) // 2] = 1.0
    return d


def impulse_response(M, theta, taps, keep=False):
    """K_syn = F_Theta(delta) on an M x M canvas with ZERO boundary (Eq. 10;
    F_approx of Eq. 4)."""
    return chain(impulse(M), theta, taps, ZERO, keep=keep)
