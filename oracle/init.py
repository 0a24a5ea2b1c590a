"""Initialisers for Theta (FP64): radial (Eq. 6), sparse sampling (Eq. 7) and
random positions (Sec. 4.2).

Test infrastructure only (see ``oracle/__init__``).

Readings (the paper defers the step size and the sampling procedure to an
appendix that is not available):
* Radial: r_l = l * dr, o_{l,i} = r_l (cos 2 pi i / N_l, sin 2 pi i / N_l) for
  i = 1..N_l, w = 1/N_l (Eq. 6, literal: no per-layer phase).  The step size
  is chosen so that the radii sum to the target's extent R:
  dr = 2 R / (L (L + 1)), with R = min((M-1)/2, r99) and r99 the smallest
  pixel-centre distance from c whose disk holds >= 99% of the target's mass.
* Sparse sampling: support = {q : K[q] > 0.01 max K}, S = |support|,
  r = sqrt(S / (N_s pi)) (Eq. 7) with N_s the first layer's tap count.  Dart
  throwing: draw a support pixel uniformly, jitter it by U[-1/2, 1/2)^2, accept
  it if it is at least r from every accepted point; after 100 N_s consecutive
  rejections shrink r by 0.9.  Layer-1 offsets are the accepted points minus
  c, layer-1 weights are the target at the rounded points, normalised to unit
  sum.  Layers 2..L take the radial pattern with extent R' = r (final value)
  and layer indices 1..L-1.
* Random: tap i of layer l uniform in [-r_l, r_l]^2 (r_l of the radial rule),
  w = 1/N_l.
* Random draws come from the counter-based SplitMix64 stream of ``oracle.rng``
  keyed by (seed, target index).
"""
from __future__ import annotations

import math

import numpy as np

from .rng import Stream, target_key


def r99(target):
    """Smallest pixel-centre distance from the centre whose closed disk holds
    at least 99% of the target's total mass (FP64)."""
    K = np.asarray(target, dtype=np.float64)
    M = K.shape[0]
    h = (M - 1) // 2
    y, x = np.mgrid[0:M, 0:M]
    d2 = ((x - h) ** 2 + (y - h) ** 2).reshape(-1)
    k = K.reshape(-1)
    total = k.sum()
    order = np.argsort(d2, kind="stable")
    d2s = d2[order]
    cum = np.cumsum(k[order])
    # last index of each distinct d2 value (a closed disk takes all ties)
    last = np.nonzero(np.r_[d2s[1:] != d2s[:-1], True])[0]
    hit = np.nonzero(cum[last] >= 0.99 * total)[0]
    idx = last[hit[0]] if len(hit) else last[-1]
    return math.sqrt(float(d2s[idx]))


def radial_extent(target):
    M = np.asarray(target).shape[0]
    return min((M - 1) / 2.0, r99(target))


def radial_layers(R, taps, first_index=1):
    """Eq. 6 with dr chosen so that the radii sum to R.  Layer l (0-based) uses
    index j = l + first_index; the number of indices is len(taps)."""
    L = len(taps)
    jmax = L + first_index - 1
    jsum = (jmax * (jmax + 1) - (first_index - 1) * first_index) / 2.0
    dr = R / jsum if jsum > 0 else 0.0
    rows = []
    for l, N in enumerate(taps):
        r = (l + first_index) * dr
        for i in range(1, int(N) + 1):
            a = 2.0 * math.pi * i / N
            rows.append((r * math.cos(a), r * math.sin(a), 1.0 / N))
    return np.array(rows, dtype=np.float64).reshape(-1, 3)


def radial_init(target, taps):
    """Eq. 6 for one target: [T][3] float64."""
    return radial_layers(radial_extent(target), [int(t) for t in taps], 1)


def ss_init(target, taps, seed, index=0):
    """Sparse-sampling initialisation (Eq. 7) of the first layer, radial
    pattern for the others.  Returns (theta [T][3], final r)."""
    K = np.asarray(target, dtype=np.float64)
    M = K.shape[0]
    c = (M - 1) / 2.0
    taps = [int(t) for t in taps]
    Ns = taps[0]
    pk = K.max()
    if not pk > 0.0:
        return radial_layers((M - 1) / 2.0, taps, 1), 0.0
    ys, xs = np.nonzero(K > 0.01 * pk)         # row-major enumeration
    S = len(xs)
    r = math.sqrt(S / (Ns * math.pi))
    st = Stream(target_key(seed, index))
    acc = []
    rejections = 0
    while len(acc) < Ns:
        j = min(int(st.uniform() * S), S - 1)
        px = float(xs[j]) + (st.uniform() - 0.5)
        py = float(ys[j]) + (st.uniform() - 0.5)
        r2 = r * r
        ok = True
        for ax, ay in acc:
            dx = px - ax
            dy = py - ay
            if dx * dx + dy * dy < r2:
                ok = False
                break
        if ok:
            acc.append((px, py))
            rejections = 0
        else:
            rejections += 1
            if rejections >= 100 * Ns:
                r = 0.9 * r
                rejections = 0
    rows = []
    wts = []
    for px, py in acc:
        rx = min(max(int(math.floor(px + 0.5)), 0), M - 1)
        ry = min(max(int(math.floor(py + 0.5)), 0), M - 1)
        rows.append((px - c, py - c))
        wts.append(K[ry, rx])
    wsum = sum(wts)
    first = np.array([(ox, oy, (w / wsum) if wsum > 0 else 1.0 / Ns)
                      for (ox, oy), w in zip(rows, wts)], dtype=np.float64)
    if len(taps) == 1:
        return first, r
    rest = radial_layers(r, taps[1:], 1)
    return np.concatenate([first, rest], axis=0), r


def random_init(target, taps, seed, index=0):
    """Random positions (Sec. 4.2 baseline): tap i of layer l uniform in
    [-r_l, r_l]^2 with r_l the radial rule's radius, w = 1/N_l."""
    taps = [int(t) for t in taps]
    R = radial_extent(target)
    L = len(taps)
    dr = 2.0 * R / (L * (L + 1))
    st = Stream(target_key(seed, index))
    rows = []
    for l, N in enumerate(taps):
        r = (l + 1) * dr
        for _ in range(N):
            ox = (2.0 * st.uniform() - 1.0) * r
            oy = (2.0 * st.uniform() - 1.0) * r
            rows.append((ox, oy, 1.0 / N))
    return np.array(rows, dtype=np.float64)
