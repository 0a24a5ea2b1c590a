"""Pins of the FP64 oracle's sparse layer, chain and impulse response
(Sec. 3.2, Eq. 2-4, Eq. 10) against closed forms, library routines,
invariants and brute force."""
import os

import numpy as np
import pytest
import scipy.ndimage as ndi
import scipy.signal as sig

from oracle import sparse as S
from synth import random_theta, uniform_image

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_bilinear_hand_values():
    X = np.array([[1, 2, 4], [8, 16, 32], [64, 128, 256]], dtype=np.float64)
    rows = [l.split() for l in open(os.path.join(GOLD, "bilinear_hand.txt")) if l[0] != "#"]
    for sx, sy, b, want in rows:
        got = S.bilinear(X, np.array(float(sx)), np.array(float(sy)), int(b))
        assert got == float(want), (sx, sy, b, got, want)


@pytest.mark.parametrize("boundary,mode", [(S.ZERO, "grid-constant"), (S.CLAMP, "nearest")])
def test_bilinear_matches_scipy_map_coordinates(boundary, mode):
    g = np.random.default_rng(11)
    X = g.random((17, 23))
    sx = g.uniform(-4, 27, size=(40, 9))
    sy = g.uniform(-4, 21, size=(40, 9))
    got = S.bilinear(X, sx, sy, boundary)
    ref = ndi.map_coordinates(X, [sy, sx], order=1, mode=mode, cval=0.0, prefilter=False)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-14)


def test_integer_taps_scatter_exactly():
    """An integer-offset layer applied to the impulse puts w_i exactly at c + o_i."""
    g = np.random.default_rng(3)
    M = 15
    c = (M - 1) // 2
    N = 9
    th = np.zeros((N, 3))
    th[:, 0] = g.integers(-6, 7, N)
    th[:, 1] = g.integers(-6, 7, N)
    th[:, 2] = g.uniform(-1, 1, N)
    K = S.impulse_response(M, th, [N])
    want = np.zeros((M, M))
    for ox, oy, w in th:
        want[c + int(oy), c + int(ox)] += w
    assert np.array_equal(K, want)
    # the same holds for FP32-rounded parameters (integers and weights are exact)
    th32 = th.astype(np.float32).astype(np.float64)
    want32 = np.zeros((M, M))
    for ox, oy, w in th32:
        want32[c + int(oy), c + int(ox)] += w
    assert np.array_equal(S.impulse_response(M, th32, [N]), want32)


def _per_layer_responses(theta, taps, m):
    return [S.impulse_response(m, lay, [len(lay)]) for lay in S.split_layers(theta, taps)]


def test_chain_is_convolution_of_layer_responses():
    taps = [5, 4, 6]
    th = random_theta(taps, 3.0, seed=5).astype(np.float64)
    m = 9                                   # each layer fits in a 9x9 window (|o| <= 3)
    Ks = _per_layer_responses(th, taps, m)
    full = Ks[0]
    for K in Ks[1:]:
        full = sig.convolve2d(full, K, mode="full")
    M = 41
    K = S.impulse_response(M, th, taps)
    c = (M - 1) // 2
    h = (full.shape[0] - 1) // 2
    crop = K[c - h:c + h + 1, c - h:c + h + 1]
    np.testing.assert_allclose(crop, full, rtol=0, atol=1e-13 * np.abs(full).max())
    outside = K.copy()
    outside[c - h:c + h + 1, c - h:c + h + 1] = 0
    assert np.abs(outside).max() == 0.0


def test_sum_is_product_of_weight_sums_and_cumulants_add():
    taps = [6, 8, 5, 7]
    th = random_theta(taps, 3.5, seed=9).astype(np.float64)
    M = 51
    K = S.impulse_response(M, th, taps)
    lays = S.split_layers(th, taps)
    Ws = [lay[:, 2].sum() for lay in lays]
    assert abs(K.sum() - np.prod(Ws)) <= 1e-14 * abs(np.prod(Ws))
    c = (M - 1) // 2
    y, x = np.mgrid[0:M, 0:M]
    Kn = K / K.sum()
    mean_x = (Kn * (x - c)).sum()
    mean_y = (Kn * (y - c)).sum()
    var_x = (Kn * (x - c - mean_x) ** 2).sum()
    var_y = (Kn * (y - c - mean_y) ** 2).sum()
    mx = my = vx = vy = 0.0
    for lay in lays:
        w = lay[:, 2]
        Wl = w.sum()
        fx = lay[:, 0] - np.floor(lay[:, 0])
        fy = lay[:, 1] - np.floor(lay[:, 1])
        lmx = (w * lay[:, 0]).sum() / Wl
        lmy = (w * lay[:, 1]).sum() / Wl
        mx += lmx
        my += lmy
        vx += (w * (lay[:, 0] ** 2 + fx * (1 - fx))).sum() / Wl - lmx ** 2
        vy += (w * (lay[:, 1] ** 2 + fy * (1 - fy))).sum() / Wl - lmy ** 2
    np.testing.assert_allclose([mean_x, mean_y, var_x, var_y], [mx, my, vx, vy], rtol=1e-12, atol=1e-12)


def test_constant_image_clamp_scales_by_weight_sums():
    taps = [5, 5, 3]
    th = random_theta(taps, 6.0, seed=2).astype(np.float64)
    X = np.full((2, 13, 19), 0.37)
    Y = S.chain(X, th, taps, S.CLAMP)
    Ws = np.prod([lay[:, 2].sum() for lay in S.split_layers(th, taps)])
    np.testing.assert_allclose(Y, 0.37 * Ws, rtol=1e-14)


def _layer_matrix(layer, H, W, boundary):
    A = np.zeros((H * W, H * W))
    for j in range(H * W):
        e = np.zeros(H * W)
        e[j] = 1.0
        A[:, j] = S.sparse_layer(e.reshape(H, W), layer, boundary).reshape(-1)
    return A


@pytest.mark.parametrize("boundary", [S.ZERO, S.CLAMP])
def test_brute_force_operator_matrices(boundary):
    """Tiny canvases: the layer is the explicit linear map whose entries are
    the bilinear corner weights; the chain is the product of those maps."""
    H, W = 7, 9
    taps = [3, 4]
    th = random_theta(taps, 2.5, seed=4).astype(np.float64)
    lays = S.split_layers(th, taps)
    # entries written from the definition: pixel p reads corners of p - o
    A = [np.zeros((H * W, H * W)) for _ in lays]
    for li, lay in enumerate(lays):
        for y in range(H):
            for x in range(W):
                for ox, oy, w in lay:
                    sx, sy = x - ox, y - oy
                    x0, y0 = int(np.floor(sx)), int(np.floor(sy))
                    fx, fy = sx - x0, sy - y0
                    for dy, dx, cw in ((0, 0, (1 - fx) * (1 - fy)), (0, 1, fx * (1 - fy)),
                                       (1, 0, (1 - fx) * fy), (1, 1, fx * fy)):
                        yy, xx = y0 + dy, x0 + dx
                        if boundary == S.CLAMP:
                            yy, xx = min(max(yy, 0), H - 1), min(max(xx, 0), W - 1)
                        elif not (0 <= yy < H and 0 <= xx < W):
                            continue
                        A[li][y * W + x, yy * W + xx] += w * cw
    for li, lay in enumerate(lays):
        np.testing.assert_allclose(_layer_matrix(lay, H, W, boundary), A[li], rtol=0, atol=1e-15)
    X = uniform_image(H, W, 1, seed=8)[0].astype(np.float64)
    want = A[1] @ (A[0] @ X.reshape(-1))
    np.testing.assert_allclose(S.chain(X, th, taps, boundary).reshape(-1), want, rtol=0, atol=1e-14)
