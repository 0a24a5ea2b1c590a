"""Filter-space interpolation (Eq. 8, Eq. 9) in FP64.

Test infrastructure only (see ``oracle/__init__``).

The basis is an ordered set of complete parameter sets f_k = Theta_k (every
entry shares the same layer and tap structure), sampled at parameter values
p_1 < ... < p_G.  This oracle takes the nodes evenly spaced on [0, 1]:
p_k = (k - 1) / (G - 1).  The paper fixes only convexity of the weights
(sum alpha = 1, alpha >= 0, Eq. 9); the reading used is the piecewise-linear
hat basis in 1-D and its tensor product in 2-D, with P clamped to [0, 1]:
    u = clamp(P, 0, 1) (G - 1),  k = min(floor(u), G - 2),  t = u - k,
    alpha_k = 1 - t,  alpha_{k+1} = t   (G = 1: alpha_1 = 1).
Offsets and weights are interpolated elementwise (Sec. 4.3).
"""
from __future__ import annotations

import numpy as np


def decode(P, G):
    """(k, t) per pixel for a G-entry axis."""
    P = np.asarray(P, dtype=np.float64)
    if G == 1:
        return np.zeros(P.shape, np.int64), np.zeros(P.shape)
    u = np.clip(P, 0.0, 1.0) * (G - 1)
    k = np.minimum(np.floor(u), G - 2)
    return k.astype(np.int64), u - k


def alpha_1d(P, G):
    """Dense interpolation weights alpha [..., G] (Eq. 9) for a 1-D basis."""
    k, t = decode(P, G)
    a = np.zeros(np.shape(P) + (G,))
    np.put_along_axis(a, k[..., None], (1.0 - t)[..., None], axis=-1)
    if G > 1:
        kk = np.minimum(k + 1, G - 1)
        prev = np.take_along_axis(a, kk[..., None], axis=-1)
        np.put_along_axis(a, kk[..., None], prev + t[..., None], axis=-1)
    return a


def alpha_2d(P0, P1, G0, G1):
    """Dense weights [..., G0*G1] (entry index i0*G1 + i1): tensor product of
    the 1-D hat weights."""
    a0 = alpha_1d(P0, G0)
    a1 = alpha_1d(P1, G1)
    return (a0[..., :, None] * a1[..., None, :]).reshape(np.shape(P0) + (G0 * G1,))


def combine(basis, alpha):
    """f = sum_k alpha_k f_k (Eq. 9).  basis: [G][T][3]; alpha: [..., G].
    Returns [..., T, 3]."""
    basis = np.asarray(basis, dtype=np.float64)
    return np.tensordot(np.asarray(alpha, np.float64), basis, axes=([-1], [0]))


def tap_field(basis, P, grid, tap):
    """Per-pixel (ox, oy, w) of one tap: the elementwise convex combination of
    the basis entries that carry non-zero weight (at most 2 in 1-D, 4 in 2-D).
    basis: [G][T][3]; P: [dims][H][W]; returns three [H][W] arrays."""
    basis = np.asarray(basis, dtype=np.float64)
    P = np.asarray(P, dtype=np.float64)
    if len(grid) == 1:
        G = grid[0]
        k, t = decode(P[0], G)
        a = basis[k, tap]                       # [H][W][3]
        if G == 1:
            v = a
        else:
            b = basis[np.minimum(k + 1, G - 1), tap]
            v = (1.0 - t)[..., None] * a + t[..., None] * b
    else:
        G0, G1 = grid
        k0, s = decode(P[0], G0)
        k1, t = decode(P[1], G1)
        k0b = np.minimum(k0 + 1, G0 - 1)
        k1b = np.minimum(k1 + 1, G1 - 1)
        v = (((1 - s) * (1 - t))[..., None] * basis[k0 * G1 + k1, tap]
             + (s * (1 - t))[..., None] * basis[k0b * G1 + k1, tap]
             + ((1 - s) * t)[..., None] * basis[k0 * G1 + k1b, tap]
             + (s * t)[..., None] * basis[k0b * G1 + k1b, tap])
    return v[..., 0], v[..., 1], v[..., 2]


def rotate_basis(base, angles):
    """Angle axis of a 2-D basis (angle-driven effects of Sec. 5): entry
    (i0, i1) is base entry i0 with every offset rotated by angles[i1]
    (counter-clockwise in (x, y)); weights unchanged.  Returns [G0 * G1][T][3]."""
    base = np.asarray(base, dtype=np.float64)
    out = []
    for b in base:
        for a in angles:
            c, s = np.cos(a), np.sin(a)
            r = b.copy()
            r[:, 0] = c * b[:, 0] - s * b[:, 1]
            r[:, 1] = s * b[:, 0] + c * b[:, 1]
            out.append(r)
    return np.stack(out)
