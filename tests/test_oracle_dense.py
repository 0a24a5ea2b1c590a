"""Pins of the dense convolution reference (Eq. 1, uniform and spatially
varying): closed-form Gaussian convolution, the impulse, scipy, and the
orientation shared with the sparse chain."""
import numpy as np
import scipy.signal as sig

from oracle import dense as D
from oracle import sparse as S
from synth import uniform_image, random_theta, disk_kernel


def _g(x, y, s2):
    return np.exp(-(x * x + y * y) / (2 * s2)) / (2 * np.pi * s2)


def test_gaussian_conv_gaussian_closed_form():
    s1, s2 = 2.0, 2.5
    n = 81
    c = n // 2
    y, x = np.mgrid[0:n, 0:n] - c
    img = _g(x, y, s1 * s1)
    h = 24
    q = np.arange(-h, h + 1)
    K = _g(q[None, :], q[:, None], s2 * s2)
    out = D.dense_uniform(img, K, rows=slice(c - 6, c + 7), cols=slice(c - 6, c + 7))
    yy, xx = np.mgrid[-6:7, -6:7]
    want = _g(xx, yy, s1 * s1 + s2 * s2)
    np.testing.assert_allclose(out, want, rtol=1e-12, atol=0)


def test_impulse_gives_kernel_orientation():
    K = np.random.default_rng(0).random((7, 7))          # non-symmetric
    img = np.zeros((21, 21))
    img[9, 12] = 1.0
    out = D.dense_uniform(img, K)
    # mass of K[q] lands at p0 + q
    np.testing.assert_array_equal(out[6:13, 9:16], K)


def test_matches_scipy_convolve2d_on_edge_padded_input():
    img = uniform_image(23, 29, 1, seed=3)[0].astype(np.float64)
    K = np.random.default_rng(2).random((9, 9))
    ref = sig.convolve2d(np.pad(img, 4, mode="edge"), K, mode="valid")
    np.testing.assert_allclose(D.dense_uniform(img, K), ref, rtol=1e-13)


def test_sparse_chain_equals_dense_conv_with_its_impulse_response_in_interior():
    taps = [5, 6]
    th = random_theta(taps, 3.0, seed=12).astype(np.float64)
    M = 17
    K = S.impulse_response(M, th, taps)
    img = uniform_image(40, 44, 1, seed=6)[0].astype(np.float64)
    a = S.chain(img, th, taps, S.CLAMP)
    b = D.dense_uniform(img, K)
    m = 10      # interior: no clamped read anywhere in the support
    np.testing.assert_allclose(a[m:-m, m:-m], b[m:-m, m:-m], rtol=0, atol=1e-14)


def test_dense_sv_constant_map_is_uniform_disk():
    img = uniform_image(30, 30, 2, seed=8).astype(np.float64)
    P = np.full((1, 30, 30), 0.25)
    cov = D.disk_coverage(lambda p: 2.0 + 30.0 * p)        # r = 9.5
    out = D.dense_sv(img, cov, P, half=11, rows=slice(5, 25), cols=slice(3, 27))
    K = disk_kernel(9.5, 23)
    ref = D.dense_uniform(img, K, rows=slice(5, 25), cols=slice(3, 27))
    np.testing.assert_allclose(out, ref, rtol=1e-12)


def test_dense_sv_uses_each_pixels_kernel():
    img = uniform_image(25, 25, 1, seed=4)[0].astype(np.float64)
    P = np.random.default_rng(3).random((1, 25, 25))
    cov = D.disk_coverage(lambda p: 1.0 + 4.0 * p)
    out = D.dense_sv(img, cov, P, half=6)
    for (y, x) in [(0, 0), (12, 12), (3, 20), (24, 7)]:
        K = disk_kernel(1.0 + 4.0 * P[0, y, x], 13)
        ref = D.dense_uniform(img, K, rows=slice(y, y + 1), cols=slice(x, x + 1))
        assert abs(out[y, x] - ref[0, 0]) < 1e-13


def _coverage_grid(cov, P, h):
    q = np.arange(-h, h + 1)
    return np.array([[float(np.ravel(cov(P, qx, qy))[0]) for qx in q] for qy in q])


def test_ellipse_coverage_reduces_to_the_disk_at_unit_aspect():
    """At aspect a = 1 both semi-axes equal r, the ray distance to the boundary
    is |q| - r, and the elliptical coverage is the disk's clamp(r + 1/2 - |q|)."""
    for r in (2.0, 5.3, 11.75, 24.0):
        P = np.array([[r], [1.0]])
        e = _coverage_grid(D.ellipse_coverage(lambda p: p, lambda p: p), P, 27)
        d = _coverage_grid(D.disk_coverage(lambda p: p), P[:1], 27)
        np.testing.assert_allclose(e, d, rtol=0, atol=1e-12)


def test_ellipse_coverage_axes_mass_and_second_moments():
    """Semi-axes (r sqrt(a), r / sqrt(a)): along the x axis the coverage is a
    1-D disk of radius r sqrt(a), along y one of radius r / sqrt(a); the mass
    approaches the area pi r^2 (area-preserving); the second moments have the
    ratio E[qx^2] / E[qy^2] = a^2 of a uniform ellipse.  Swapping the axes or
    mis-scaling the boundary distance fails each of these."""
    r, a = 9.0, 2.0
    ax, ay = r * np.sqrt(a), r / np.sqrt(a)
    P = np.array([[r], [a]])
    h = 20
    K = _coverage_grid(D.ellipse_coverage(lambda p: p, lambda p: p), P, h)
    q = np.arange(-h, h + 1)
    np.testing.assert_allclose(K[h, :], np.clip(ax + 0.5 - np.abs(q), 0, 1), atol=1e-12)
    np.testing.assert_allclose(K[:, h], np.clip(ay + 0.5 - np.abs(q), 0, 1), atol=1e-12)
    assert abs(K.sum() / (np.pi * r * r) - 1.0) < 0.01
    qy, qx = np.mgrid[-h:h + 1, -h:h + 1]
    ratio = (K * qx * qx).sum() / (K * qy * qy).sum()
    assert abs(ratio / (a * a) - 1.0) < 0.03
