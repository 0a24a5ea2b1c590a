"""Learned initialiser (an extension, not in the paper): a small conv encoder
plus MLP that maps a target kernel to a starting Theta for the optimiser of
Sec. 4.4, in FP64 on BF16-rounded operands.

Test infrastructure only (see ``oracle/__init__``).

Network (input 64 x 64 x 1):
    6 x [conv 3x3, stride 2, zero padding 1, + bias, ReLU], widths 32, 64,
    128, 128, 256, 256 (spatial 64 -> 32 -> 16 -> 8 -> 4 -> 2 -> 1),
    FC 256 -> 512 + ReLU, FC 512 -> 144.
The 144 outputs are Theta of 4 layers x 12 taps, tap t at (3t, 3t+1, 3t+2) =
(o_x / hw, o_y / hw, w), where hw is the scale of the input grid (below).

Precision model (the definition both sides follow):
* every layer's operands (its input activations and its weights) are rounded
  to BF16 (round to nearest even) before the contraction; the contraction
  itself and the bias add are exact here (FP32 accumulation on the device);
* a hidden layer's output is ReLU(z) rounded first to FP32, then to BF16, so
  that the rounding decision is taken from the same FP32 value as on the
  device; the last layer's output is z (no rounding);
* backward: g = dL/dz of a layer is rounded to FP32; the bias gradient is the
  plain sum of g; g rounded to BF16 enters both contractions (weight
  gradient against the layer's BF16 input, input gradient against the BF16
  weights); the input gradient times [input > 0] is the previous layer's g.
  The weight gradient is taken as the gradient of the FP32 master weights.
* loss: mean over B x 144 of (y_hat - y)^2.

Input preparation: the target (M x M, M odd, centre c = (M-1)/2, pixel y
covering [y - 1/2, y + 1/2]) is resampled by exact area averaging onto 64 x 64
cells of side s = max(1, M / 64) centred on c (cell i spans
[c + (i - 32) s, c + (i - 31) s]); the result is divided by its maximum and
rounded to BF16.  Offsets in target pixels are o = (network output) x hw with
hw = 32 s.

``exact=True`` switches every rounding off (used by the finite-difference
pins).
"""
from __future__ import annotations

import numpy as np

WIDTHS = (32, 64, 128, 128, 256, 256)
FC = (512, 144)
IN_SIDE = 64
OUT_TAPS = 48


def arch():
    """Layer list: ('conv', cin, cout) x 6, ('fc', fin, fout) x 2."""
    layers, cin = [], 1
    for w in WIDTHS:
        layers.append(("conv", cin, w))
        cin = w
    layers.append(("fc", cin, FC[0]))
    layers.append(("fc", FC[0], FC[1]))
    return layers


def param_shapes(layers=None):
    """(weight shape, bias shape) per layer in PyTorch layout."""
    out = []
    for kind, a, b in layers or arch():
        out.append(((b, a, 3, 3) if kind == "conv" else (b, a), (b,)))
    return out


def param_count(layers=None):
    return int(sum(np.prod(w) + np.prod(b) for w, b in param_shapes(layers)))


def unflatten(flat, layers=None):
    """Flat parameter vector (order W1, b1, W2, b2, ...) -> list of (W, b)."""
    flat = np.asarray(flat, dtype=np.float64)
    out, o = [], 0
    for ws, bs in param_shapes(layers):
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        out.append((flat[o:o + nw].reshape(ws), flat[o + nw:o + nw + nb].reshape(bs)))
        o += nw + nb
    assert o == flat.size
    return out


def flatten(pairs):
    return np.concatenate([np.concatenate([W.reshape(-1), b.reshape(-1)]) for W, b in pairs])


# ---------------------------------------------------------------------------
# rounding
# ---------------------------------------------------------------------------
def to_f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def to_bf16(x):
    """Round to FP32, then to BF16 with round-to-nearest-even (finite inputs);
    returns the BF16 values as float64."""
    u = np.asarray(x, dtype=np.float64).astype(np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------------------
# input preparation
# ---------------------------------------------------------------------------
def area_matrix(M, n=IN_SIDE):
    """A[i][y] = |cell i  intersect  pixel y| / s (cells of side s centred on c)."""
    s = max(1.0, M / n)
    c = (M - 1) / 2.0
    A = np.zeros((n, M))
    for i in range(n):
        lo, hi = c + (i - n // 2) * s, c + (i - n // 2 + 1) * s
        for y in range(M):
            ov = min(hi, y + 0.5) - max(lo, y - 0.5)
            if ov > 0:
                A[i, y] = ov / s
    return A, s


def prepare_input(target, exact=False):
    """Target [M][M] -> (x [64][64] (BF16 values unless exact), hw)."""
    K = np.asarray(target, dtype=np.float64)
    A, s = area_matrix(K.shape[0])
    x = A @ K @ A.T
    pk = x.max()
    if pk > 0:
        x = x / pk
    return (x if exact else to_bf16(x)), IN_SIDE // 2 * s


# ---------------------------------------------------------------------------
# layers
# ---------------------------------------------------------------------------
def im2col(x):
    """x [B][C][H][W] -> columns [B][Ho][Wo][C][3][3] of the stride-2,
    padding-1 3x3 window (out-of-range reads are 0)."""
    B, C, H, W = x.shape
    Ho, Wo = (H + 1) // 2, (W + 1) // 2
    xp = np.zeros((B, C, H + 2, W + 2))
    xp[:, :, 1:H + 1, 1:W + 1] = x
    cols = np.zeros((B, Ho, Wo, C, 3, 3))
    for ky in range(3):
        for kx in range(3):
            cols[:, :, :, :, ky, kx] = xp[:, :, ky:ky + 2 * Ho:2, kx:kx + 2 * Wo:2].transpose(0, 2, 3, 1)
    return cols


def col2im(dcols, shape):
    """Transpose of im2col: sums every column entry back onto its input pixel."""
    B, C, H, W = shape
    Ho, Wo = dcols.shape[1], dcols.shape[2]
    dxp = np.zeros((B, C, H + 2, W + 2))
    for ky in range(3):
        for kx in range(3):
            dxp[:, :, ky:ky + 2 * Ho:2, kx:kx + 2 * Wo:2] += dcols[:, :, :, :, ky, kx].transpose(0, 3, 1, 2)
    return dxp[:, :, 1:H + 1, 1:W + 1]


def forward(flat, x, layers=None, exact=False):
    """x [B][64][64] (the prepared inputs).  Returns (y_hat [B][144], cache)."""
    rb = (lambda v: v) if exact else to_bf16
    r32 = (lambda v: v) if exact else to_f32
    lays = layers or arch()
    params = unflatten(flat, lays)
    a = rb(np.asarray(x, dtype=np.float64))
    if a.ndim == 3:
        a = a[:, None]
    inputs = []
    for li, ((kind, cin, cout), (W, b)) in enumerate(zip(lays, params)):
        inputs.append(a)
        Wq = rb(W)
        if kind == "conv":
            cols = im2col(a)
            z = np.tensordot(cols, Wq, axes=([3, 4, 5], [1, 2, 3])) + b      # [B][Ho][Wo][cout]
            z = z.transpose(0, 3, 1, 2)
        else:
            z = a.reshape(a.shape[0], -1) @ Wq.T + b
        if li == len(lays) - 1:
            return z, {"inputs": inputs, "layers": lays}
        a = rb(r32(np.maximum(z, 0.0)))


def loss(y_hat, y):
    d = np.asarray(y_hat, dtype=np.float64) - np.asarray(y, dtype=np.float64)
    return float(np.mean(d * d))


def backward(flat, cache, y_hat, y, exact=False):
    """Gradient of the loss w.r.t. the flat parameters (same layout)."""
    rb = (lambda v: v) if exact else to_bf16
    r32 = (lambda v: v) if exact else to_f32
    lays = cache["layers"]
    params = unflatten(flat, lays)
    y_hat = np.asarray(y_hat, dtype=np.float64)
    g = r32(2.0 * (y_hat - np.asarray(y, dtype=np.float64)) / y_hat.size)
    grads = [None] * len(lays)
    for li in range(len(lays) - 1, -1, -1):
        kind, cin, cout = lays[li]
        W, _ = params[li]
        a = cache["inputs"][li]
        if kind == "conv":
            gb = g.sum(axis=(0, 2, 3))
        else:
            gb = g.sum(axis=0)
        gq = rb(g)
        Wq = rb(W)
        if kind == "conv":
            cols = im2col(a)                                   # [B][Ho][Wo][cin][3][3]
            gW = np.tensordot(gq, cols, axes=([0, 2, 3], [0, 1, 2]))     # [cout][cin][3][3]
            if li > 0:
                dcols = np.tensordot(gq.transpose(0, 2, 3, 1), Wq, axes=([3], [0]))
                gx = col2im(dcols, a.shape)
        else:
            af = a.reshape(a.shape[0], -1)
            gW = gq.T @ af
            if li > 0:
                gx = (gq @ Wq).reshape(a.shape)
        grads[li] = (gW, gb)
        if li > 0:
            g = r32(gx * (a > 0))
    return flatten(grads)


def adam(flat, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1).  Returns (flat, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return flat - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed, layers=None):
    """Kaiming-uniform weights (bound sqrt(6 / fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    pairs = []
    for ws, bs in param_shapes(layers):
        fan_in = int(np.prod(ws[1:]))
        bound = np.sqrt(6.0 / fan_in)
        pairs.append((rng.uniform(-bound, bound, ws), np.zeros(bs)))
    return flatten(pairs)


def label(theta48, hw):
    """Theta [48][3] in target pixels -> the 144 regression targets."""
    t = np.array(theta48, dtype=np.float64).reshape(OUT_TAPS, 3)
    t[:, :2] /= hw
    return t.reshape(-1)


def theta_of(y_hat_row, hw):
    """One row of network output -> Theta [48][3] in target pixels."""
    t = np.array(y_hat_row, dtype=np.float64).reshape(OUT_TAPS, 3)
    t[:, :2] *= hw
    return t
