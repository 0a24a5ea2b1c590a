"""Seeded synthetic inputs shared by the FP64 oracle and the HIP path.

This module only *draws inputs*: images, parameter maps, dense target kernels,
random sparse-complex parameters and target batches.  It contains none of the
sparse kernel complex's arithmetic (no bilinear sampling, no layer, no loss, no
optimiser, no interpolation); those live separately in ``oracle/`` (FP64, CPU)
and in the HIP library.

Every generator takes an explicit integer seed and uses numpy's PCG64 stream, so
a (function, arguments, seed) triple names one array exactly.

The paper's own evaluation images (five photographs) and its arbitrary kernels
(silhouettes, glyphs, measured PSFs) are not available; the procedural
generators below stand in for them with the same shapes and value ranges:
* images: smooth gradient noise plus step edges, values in [0, 1];
* parameter maps: low-frequency noise in [0, 1] (a blur-intensity field);
* targets: Gaussians, disks, rings, regular polygons and stars, normalised to
  unit sum, anti-aliased over one pixel.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "rng", "gradient_noise", "noise_image", "param_map", "uniform_image",
    "gaussian_kernel", "aniso_gaussian_kernel", "disk_kernel", "ellipse_kernel",
    "polygon_kernel", "ring_kernel", "star_kernel", "shape_kernel",
    "random_theta", "TargetBatch", "shape_batch", "mixed_batch", "pack_targets",
    "line_kernel", "direction_map", "pseudo_depth", "tilt_shift_map",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


# ----------------------------------------------------------------------------
# images and parameter maps
# ----------------------------------------------------------------------------
def _fade(t):
    return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)


def gradient_noise(H: int, W: int, period: float, g: np.random.Generator) -> np.ndarray:
    """One octave of 2-D gradient (Perlin-style) noise with lattice spacing
    ``period`` pixels; roughly zero-mean, |value| <= ~0.7."""
    nx = int(math.ceil(W / period)) + 2
    ny = int(math.ceil(H / period)) + 2
    ang = g.uniform(0.0, 2.0 * math.pi, size=(ny, nx))
    gxl, gyl = np.cos(ang), np.sin(ang)
    off = g.uniform(0.0, 1.0, size=2)
    ys = (np.arange(H, dtype=np.float64) + 0.5) / period + off[0]
    xs = (np.arange(W, dtype=np.float64) + 0.5) / period + off[1]
    y, x = np.meshgrid(ys, xs, indexing="ij")
    x0 = np.floor(x).astype(np.int64)
    y0 = np.floor(y).astype(np.int64)
    fx = x - x0
    fy = y - y0

    def corner(dy, dx):
        gx = gxl[y0 + dy, x0 + dx]
        gy = gyl[y0 + dy, x0 + dx]
        return gx * (fx - dx) + gy * (fy - dy)

    u, v = _fade(fx), _fade(fy)
    top = corner(0, 0) * (1 - u) + corner(0, 1) * u
    bot = corner(1, 0) * (1 - u) + corner(1, 1) * u
    return top * (1 - v) + bot * v


def _minmax(a: np.ndarray) -> np.ndarray:
    lo, hi = a.min(), a.max()
    return (a - lo) / (hi - lo) if hi > lo else np.zeros_like(a)


def noise_image(H: int, W: int, C: int = 3, seed: int = 2, octaves: int = 4,
                period: float = 128.0, persistence: float = 0.5,
                n_rects: int = 200) -> np.ndarray:
    """Float32 image [C][H][W] in [0, 1]: ``octaves`` of gradient noise (base
    period ``period`` px, amplitude ratio ``persistence``) plus ``n_rects``
    axis-aligned rectangles with amplitude U[-0.3, 0.3] (step edges), min-max
    normalised per channel."""
    g = rng(seed)
    out = np.empty((C, H, W), dtype=np.float32)
    for c in range(C):
        acc = np.zeros((H, W))
        amp, per = 1.0, period
        for _ in range(octaves):
            acc += amp * gradient_noise(H, W, per, g)
            amp *= persistence
            per /= 2.0
        for _ in range(n_rects):
            w = int(g.integers(8, max(9, W // 6)))
            h = int(g.integers(8, max(9, H // 6)))
            x = int(g.integers(-w // 2, W))
            y = int(g.integers(-h // 2, H))
            acc[max(y, 0):max(y + h, 0), max(x, 0):max(x + w, 0)] += g.uniform(-0.3, 0.3)
        out[c] = _minmax(acc)
    return out


def param_map(H: int, W: int, seed: int = 3, octaves: int = 2, period: float = 512.0,
              dims: int = 1) -> np.ndarray:
    """Float32 parameter map [dims][H][W] in [0, 1]: low-frequency gradient
    noise (``octaves`` octaves, base period ``period`` px), min-max
    normalised per dimension."""
    g = rng(seed)
    out = np.empty((dims, H, W), dtype=np.float32)
    for d in range(dims):
        acc = np.zeros((H, W))
        amp, per = 1.0, period
        for _ in range(octaves):
            acc += amp * gradient_noise(H, W, per, g)
            amp *= 0.5
            per /= 2.0
        out[d] = _minmax(acc)
    return out


def uniform_image(H: int, W: int, C: int = 1, seed: int = 1) -> np.ndarray:
    """Float32 [C][H][W] of U[0, 1) noise."""
    return rng(seed).random((C, H, W), dtype=np.float64).astype(np.float32)


# ----------------------------------------------------------------------------
# dense target kernels (all odd-sided M x M, centre at ((M-1)/2, (M-1)/2),
# row index = y, column index = x, normalised to unit sum)
# ----------------------------------------------------------------------------
def _grid(M: int):
    h = (M - 1) / 2.0
    y, x = np.mgrid[0:M, 0:M].astype(np.float64)
    return x - h, y - h


def _normalise(k: np.ndarray) -> np.ndarray:
    s = k.sum()
    return (k / s) if s > 0 else k


def gaussian_kernel(M: int, sigma: float) -> np.ndarray:
    x, y = _grid(M)
    return _normalise(np.exp(-(x * x + y * y) / (2.0 * sigma * sigma)))


def aniso_gaussian_kernel(M: int, sx: float, sy: float, rot: float) -> np.ndarray:
    x, y = _grid(M)
    c, s = math.cos(rot), math.sin(rot)
    u = c * x + s * y
    v = -s * x + c * y
    return _normalise(np.exp(-0.5 * ((u / sx) ** 2 + (v / sy) ** 2)))


def _aa(sdf: np.ndarray) -> np.ndarray:
    """Anti-aliased coverage from a signed distance (negative inside)."""
    return np.clip(0.5 - sdf, 0.0, 1.0)


def disk_kernel(r: float, M: int | None = None) -> np.ndarray:
    """Uniform disk of radius r px: clamp(r + 1/2 - |q|, 0, 1), unit sum.
    Default window side 2*ceil(r+1)+1."""
    if M is None:
        M = 2 * int(math.ceil(r + 1.0)) + 1
    x, y = _grid(M)
    return _normalise(_aa(np.hypot(x, y) - r))


def ellipse_kernel(r: float, aspect: float, M: int | None = None) -> np.ndarray:
    """Axis-aligned elliptical disk with semi-axes (r*sqrt(a), r/sqrt(a))
    (area-preserving in a), coverage from the radial distance scaled by the
    local radius; unit sum."""
    ax, ay = r * math.sqrt(aspect), r / math.sqrt(aspect)
    if M is None:
        M = 2 * int(math.ceil(max(ax, ay) + 1.0)) + 1
    x, y = _grid(M)
    rho = np.hypot(x / ax, y / ay)
    # distance to the boundary along the ray, in pixels
    scale = np.where(rho > 0, np.hypot(x, y) / np.maximum(rho, 1e-300), min(ax, ay))
    return _normalise(_aa((rho - 1.0) * scale))


def line_kernel(length: float, width: float = 1.0, M: int | None = None) -> np.ndarray:
    """Horizontal motion-blur segment of the given length (capsule of the given
    width around the centre line), anti-aliased, unit sum."""
    h = length / 2.0
    if M is None:
        M = 2 * int(math.ceil(h + width)) + 1
    x, y = _grid(M)
    dx = np.maximum(np.abs(x) - h, 0.0)
    return _normalise(_aa(np.hypot(dx, y) - width / 2.0))


def direction_map(H: int, W: int, kind: str = "radial") -> np.ndarray:
    """Two-channel parameter map for angle-driven blur: P0 = distance from the
    image centre / the corner distance; P1 = the blur direction mod pi, over
    pi: along the ray from the centre ("radial", zoom blur) or across it
    ("rotational")."""
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    dy, dx = y - (H - 1) / 2.0, x - (W - 1) / 2.0
    r = np.hypot(dx, dy)
    a = np.arctan2(dy, dx) + (0.0 if kind == "radial" else math.pi / 2.0)
    return np.stack([r / r.max(), np.mod(a, math.pi) / math.pi]).astype(np.float32)


def pseudo_depth(H: int, W: int, seed: int = 12, relief: float = 0.15, period: float = 256.0) -> np.ndarray:
    """Float64 [H][W] pseudo-depth in [0, 1]: a ground plane receding from
    the bottom row (depth 0) to the top row (depth 1), plus smooth relief
    (one octave of gradient noise, amplitude ``relief``), clipped to [0, 1]."""
    g = rng(seed)
    ramp = 1.0 - np.arange(H, dtype=np.float64)[:, None] / max(H - 1, 1)
    d = ramp + relief * gradient_noise(H, W, period, g) / 0.7
    return np.clip(d, 0.0, 1.0)


def tilt_shift_map(H: int, W: int, focus: float = 0.5, depth_of_field: float = 0.08, falloff: float = 0.35,
                   seed: int = 12) -> np.ndarray:
    """Parameter map [1][H][W] of a tilt-shift effect: zero blur within
    ``depth_of_field`` of the focal depth, growing linearly with the
    pseudo-depth distance beyond it and saturating at ``falloff``."""
    d = pseudo_depth(H, W, seed)
    b = np.clip((np.abs(d - focus) - depth_of_field) / falloff, 0.0, 1.0)
    return b[None].astype(np.float32)


def _polygon_sdf(x, y, n: int, R: float, rot: float):
    """Signed distance to a regular n-gon with circumradius R."""
    ang = np.arctan2(y, x) - rot
    seg = 2.0 * math.pi / n
    a = np.mod(ang, seg) - seg / 2.0
    r = np.hypot(x, y)
    apothem = R * math.cos(math.pi / n)
    return r * np.cos(a) - apothem


def polygon_kernel(M: int, n: int, R: float, rot: float = 0.0) -> np.ndarray:
    x, y = _grid(M)
    return _normalise(_aa(_polygon_sdf(x, y, n, R, rot)))


def ring_kernel(M: int, R: float, inner: float) -> np.ndarray:
    """Annulus with outer radius R and inner radius inner*R."""
    x, y = _grid(M)
    r = np.hypot(x, y)
    sdf = np.maximum(r - R, inner * R - r)
    return _normalise(_aa(sdf))


def star_kernel(M: int, points: int, R: float, inner: float, rot: float = 0.0) -> np.ndarray:
    """Star polygon with ``points`` tips at radius R and valleys at inner*R.
    Coverage is estimated on a 4x4 supersampled grid of each pixel."""
    n = 4
    acc = np.zeros((M, M))
    x, y = _grid(M)
    ri = inner * R
    verts = []
    for k in range(2 * points):
        rad = R if k % 2 == 0 else ri
        th = rot + math.pi * k / points
        verts.append((rad * math.cos(th), rad * math.sin(th)))
    verts = np.array(verts)
    for sy in range(n):
        for sx in range(n):
            px = x + (sx + 0.5) / n - 0.5
            py = y + (sy + 0.5) / n - 0.5
            inside = np.zeros_like(px, dtype=bool)
            j = len(verts) - 1
            for i in range(len(verts)):
                xi, yi = verts[i]
                xj, yj = verts[j]
                cond = ((yi > py) != (yj > py)) & (
                    px < (xj - xi) * (py - yi) / ((yj - yi) if yj != yi else 1e-300) + xi)
                inside ^= cond
                j = i
            acc += inside
    return _normalise(acc / (n * n))


SHAPES = ("hexagon", "pentagon", "ring", "star", "gaussian")


def shape_kernel(kind: str, M: int, g: np.random.Generator) -> tuple[np.ndarray, dict]:
    """One procedural target of side M with randomised parameters; returns
    (kernel, params)."""
    R = 0.9 * (M - 1) / 2.0
    rot = float(g.uniform(0.0, 2.0 * math.pi))
    if kind == "hexagon":
        return polygon_kernel(M, 6, R, rot), {"kind": kind, "R": R, "rot": rot}
    if kind == "pentagon":
        return polygon_kernel(M, 5, R, rot), {"kind": kind, "R": R, "rot": rot}
    if kind == "ring":
        inner = float(g.uniform(0.4, 0.8))
        return ring_kernel(M, R, inner), {"kind": kind, "R": R, "inner": inner}
    if kind == "star":
        pts = int(g.integers(5, 9))
        inner = float(g.uniform(0.35, 0.55))
        return star_kernel(M, pts, R, inner, rot), {"kind": kind, "R": R, "points": pts,
                                                     "inner": inner, "rot": rot}
    if kind == "gaussian":
        sx, sy = float(g.uniform(1.0, 20.0)), float(g.uniform(1.0, 20.0))
        r2 = float(g.uniform(0.0, math.pi))
        return aniso_gaussian_kernel(M, sx, sy, r2), {"kind": kind, "sx": sx, "sy": sy, "rot": r2}
    raise ValueError(kind)


# ----------------------------------------------------------------------------
# random sparse-complex parameters (for parity tests; not an initialiser)
# ----------------------------------------------------------------------------
def random_theta(taps, radius: float, seed: int, weight_range=(0.02, 0.3),
                 dtype=np.float32) -> np.ndarray:
    """Random [T][3] = (ox, oy, w) rows, layer-major, offsets uniform in a
    disk of ``radius`` pixels, weights uniform in ``weight_range``."""
    g = rng(seed)
    T = int(sum(taps))
    r = radius * np.sqrt(g.random(T))
    a = g.uniform(0.0, 2.0 * math.pi, T)
    th = np.empty((T, 3), dtype=np.float64)
    th[:, 0] = r * np.cos(a)
    th[:, 1] = r * np.sin(a)
    th[:, 2] = g.uniform(weight_range[0], weight_range[1], T)
    return th.astype(dtype)


# ----------------------------------------------------------------------------
# target batches
# ----------------------------------------------------------------------------
@dataclass
class TargetBatch:
    kernels: list            # list of float32 [M][M]
    L: np.ndarray            # int32 [B]
    taps: list               # list of int32 arrays (per-target layer tap counts)
    params: list             # generator parameters per target

    @property
    def B(self) -> int:
        return len(self.kernels)


def shape_batch(B: int, M: int, L: int, N: int, seed: int,
                kinds=("hexagon", "pentagon", "ring", "star")) -> TargetBatch:
    """B targets of one side M, shapes drawn with equal probability from
    ``kinds``; every target uses L layers of N taps."""
    g = rng(seed)
    ks, ps = [], []
    for _ in range(B):
        kind = kinds[int(g.integers(0, len(kinds)))]
        k, p = shape_kernel(kind, M, g)
        ks.append(k.astype(np.float32))
        ps.append(p)
    return TargetBatch(ks, np.full(B, L, np.int32), [np.full(L, N, np.int32)] * B, ps)


def mixed_batch(B: int, seed: int, side=(15, 127), layers=(2, 6), taps=(6, 16),
                kinds=SHAPES, fixed_L: int | None = None, fixed_N: int | None = None) -> TargetBatch:
    """Uneven batch: odd side uniform over [side], L uniform over [layers],
    N uniform over [taps] (one N per target, held for all its layers), shape
    family uniform over ``kinds``."""
    g = rng(seed)
    odd = np.arange(side[0] | 1, side[1] + 1, 2)
    ks, Ls, Ts, ps = [], [], [], []
    for _ in range(B):
        M = int(odd[int(g.integers(0, len(odd)))])
        kind = kinds[int(g.integers(0, len(kinds)))]
        k, p = shape_kernel(kind, M, g)
        L = fixed_L if fixed_L is not None else int(g.integers(layers[0], layers[1] + 1))
        N = fixed_N if fixed_N is not None else int(g.integers(taps[0], taps[1] + 1))
        p.update({"M": M, "L": L, "N": N})
        ks.append(k.astype(np.float32))
        Ls.append(L)
        Ts.append(np.full(L, N, np.int32))
        ps.append(p)
    return TargetBatch(ks, np.array(Ls, np.int32), Ts, ps)


def pack_targets(batch: TargetBatch):
    """Flatten a batch into the packed layout used by the batched optimiser:
    returns (desc int32 [B][5] = (side, L, taps_off, theta_off, target_off),
    taps int32 [sum L], targets float32 [sum M^2])."""
    B = batch.B
    desc = np.zeros((B, 5), np.int32)
    taps_all, tgt_all = [], []
    to = th = tg = 0
    for b in range(B):
        M = batch.kernels[b].shape[0]
        L = int(batch.L[b])
        desc[b] = (M, L, to, th, tg)
        taps_all.append(np.asarray(batch.taps[b], np.int32))
        tgt_all.append(batch.kernels[b].reshape(-1))
        to += L
        th += int(np.sum(batch.taps[b]))
        tg += M * M
    return desc, np.concatenate(taps_all), np.concatenate(tgt_all).astype(np.float32)
