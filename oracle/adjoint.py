"""Gradients of the sparse chain (FP64): the end-to-end differentiation of
Sec. 4.1 (all offsets and weights of all layers are learned jointly), written
as an explicit adjoint of the forward pass in ``oracle.sparse``.

Test infrastructure only (see ``oracle/__init__``).

For one layer with input X = X_{l-1}, output gradient G = dL/dX_l and a tap
(o, w):
* dL/dw      = sum_p G[p] * B(X, p - o)
* dL/do_x    = -w * sum_p G[p] * dB/ds_x(X, s)|_{s = p - o}   (likewise y),
  with dB/ds_x = (1-fy)(X[y0,x0+1] - X[y0,x0]) + fy(X[y0+1,x0+1] - X[y0+1,x0])
  (floor makes it right-continuous at integer positions; x0 = p + floor(-o)
  exactly, so the side of a kink is the same at every pixel);
* dL/dX_{l-1} is the exact transpose of the gather: every output pixel sends
  G[p] * w * corner_weight to each of its four (boundary-mapped) corners;
  corners that fall outside a ZERO canvas send nothing, CLAMP corners send to
  the clamped pixel.
Channels share taps, so tap gradients sum over channels.
"""
from __future__ import annotations

import numpy as np

from .sparse import ZERO, CLAMP, split_layers, pixel_grid, sparse_layer
from . import loss as _loss


def _corner_index(yy, xx, H, W, boundary):
    if boundary == CLAMP:
        return np.clip(yy, 0, H - 1), np.clip(xx, 0, W - 1), np.ones(yy.shape, bool)
    inside = (yy >= 0) & (yy < H) & (xx >= 0) & (xx < W)
    return np.clip(yy, 0, H - 1), np.clip(xx, 0, W - 1), inside


def layer_vjp(X, layer, boundary, G):
    """Adjoint of one uniform sparse layer.  X: [..., H, W] input of the layer,
    G: gradient w.r.t. its output.  Returns (dlayer [N][3], dX)."""
    X = np.asarray(X, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    H, W = X.shape[-2:]
    px, py = pixel_grid(H, W)
    lead = X.shape[:-2]
    dlayer = np.zeros((len(layer), 3))
    dX = np.zeros_like(X)
    for i, (ox, oy, w) in enumerate(np.asarray(layer, dtype=np.float64)):
        # p - o with the integer part p + floor(-o) and the fraction from o
        # alone (exact; see oracle.sparse.bilinear_offset)
        flx = np.floor(-ox)
        fly = np.floor(-oy)
        fx = np.full(px.shape, -ox - flx)
        fy = np.full(py.shape, -oy - fly)
        x0 = (px + flx).astype(np.int64)
        y0 = (py + fly).astype(np.int64)
        corners = []
        for dy in (0, 1):
            for dx in (0, 1):
                yi, xi, ok = _corner_index(y0 + dy, x0 + dx, H, W, boundary)
                corners.append((yi, xi, ok, np.where(ok, X[..., yi, xi], 0.0)))
        v00, v01, v10, v11 = (c[3] for c in corners)
        B = (1 - fx) * (1 - fy) * v00 + fx * (1 - fy) * v01 + (1 - fx) * fy * v10 + fx * fy * v11
        dBx = (1 - fy) * (v01 - v00) + fy * (v11 - v10)
        dBy = (1 - fx) * (v10 - v00) + fx * (v11 - v01)
        dlayer[i, 2] = np.sum(G * B)
        dlayer[i, 0] = -w * np.sum(G * dBx)
        dlayer[i, 1] = -w * np.sum(G * dBy)
        cw = ((1 - fx) * (1 - fy), fx * (1 - fy), (1 - fx) * fy, fx * fy)
        for (yi, xi, ok, _), c in zip(corners, cw):
            contrib = np.where(ok, w * c * G, 0.0)
            flat = (yi * W + xi).reshape(-1)
            dXf = dX.reshape(lead + (H * W,))
            if lead:
                cf = contrib.reshape(lead + (H * W,))
                for idx in np.ndindex(*lead):
                    np.add.at(dXf[idx], flat, cf[idx])
            else:
                np.add.at(dXf, flat, contrib.reshape(-1))
    return dlayer, dX


def chain_vjp(X0, theta, taps, boundary, GL):
    """Reverse pass through the chain of Eq. 3.  Returns (dtheta [T][3],
    dX0) given GL = dL/dX_L."""
    layers = split_layers(theta, taps)
    Xs = [np.asarray(X0, dtype=np.float64)]
    for layer in layers[:-1]:
        Xs.append(sparse_layer(Xs[-1], layer, boundary))
    G = np.asarray(GL, dtype=np.float64)
    grads = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        grads[l], G = layer_vjp(Xs[l], layers[l], boundary, G)
    return np.concatenate(grads, axis=0), G


def impulse_loss_grad(target, theta, taps, kind=_loss.NMSE, eps=1e-3):
    """Loss of Eq. 11 (or the normalised MSE) between F_Theta(delta) and the
    target, its PSNR, and dloss/dTheta.  Returns (loss, psnr_db, dtheta)."""
    from .sparse import impulse, chain
    target = np.asarray(target, dtype=np.float64)
    M = target.shape[0]
    d = impulse(M)
    K = chain(d, theta, taps, ZERO)
    loss, gK = _loss.loss_and_grad(K, target, kind, eps)
    dtheta, _ = chain_vjp(d, theta, taps, ZERO, gK)
    return loss, _loss.psnr_db(K, target), dtheta
