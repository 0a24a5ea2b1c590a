"""Pins of the oracle's initialisers (Eq. 6, Eq. 7), the counter-based
generator, filter-space interpolation (Eq. 9) and the SV chain (Sec. 4.3)."""
import math
import os

import numpy as np
import pytest

from oracle import sparse as S
from oracle import init as I
from oracle import rng as R
from oracle import interp as IP
from oracle import svfilter as SV
from synth import gaussian_kernel, disk_kernel, ring_kernel, random_theta, noise_image, param_map

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_vector():
    want = [int(l, 16) for l in open(os.path.join(GOLD, "splitmix64_seed0.txt")) if l[0] != "#"]
    st = R.Stream(0)
    assert [st.next_u64() for _ in range(4)] == want


def test_radial_init_config1_fixture():
    """31x31 Gaussian sigma=6: r99 exceeds the half-width, so R = 15 and the
    radii are 2.5, 5, 7.5 (Eq. 6 with the radii summing to R)."""
    K = gaussian_kernel(31, 6.0)
    assert I.r99(K) > 15.0
    th = I.radial_init(K, [8, 8, 8])
    want = np.loadtxt(os.path.join(GOLD, "radial_L3N8_R15.txt"))
    np.testing.assert_allclose(th, want, rtol=0, atol=1e-14)


def test_r99_brute_force():
    for K in (disk_kernel(5.3, 21), ring_kernel(25, 10.0, 0.6), gaussian_kernel(41, 4.0)):
        M = K.shape[0]
        c = (M - 1) // 2
        y, x = np.mgrid[0:M, 0:M]
        d = np.hypot(x - c, y - c)
        best = None
        for rad in sorted(set(d.reshape(-1).tolist())):
            if K[d <= rad + 1e-12].sum() >= 0.99 * K.sum():
                best = rad
                break
        assert abs(I.r99(K) - best) < 1e-12


def test_radial_invariants():
    K = disk_kernel(9.0, 31)
    taps = [6, 9, 12, 7]
    th = I.radial_init(K, taps)
    lays = S.split_layers(th, taps)
    R_ = I.radial_extent(K)
    radii = [float(np.hypot(l[0, 0], l[0, 1])) for l in lays]
    assert abs(sum(radii) - R_) < 1e-12
    for l, lay in enumerate(lays):
        assert abs(lay[:, 2].sum() - 1.0) < 1e-15
        np.testing.assert_allclose(np.hypot(lay[:, 0], lay[:, 1]), radii[l], rtol=1e-14)
        np.testing.assert_allclose(radii[l], (l + 1) * radii[0], rtol=1e-14)
    Ksyn = S.impulse_response(31, th, taps)
    assert abs(Ksyn.sum() - 1.0) < 1e-13          # nothing leaves the canvas


def test_ss_init_properties_and_determinism():
    K = ring_kernel(41, 17.0, 0.6)
    taps = [12, 12, 12, 12]
    th, r = I.ss_init(K, taps, seed=4, index=3)
    th2, r2 = I.ss_init(K, taps, seed=4, index=3)
    assert np.array_equal(th, th2) and r == r2
    assert not np.array_equal(th, I.ss_init(K, taps, seed=4, index=4)[0])
    c = (41 - 1) / 2
    first = th[:12]
    pts = first[:, :2] + c
    sup_y, sup_x = np.nonzero(K > 0.01 * K.max())
    for px, py in pts:   # within half a pixel (per axis) of some support pixel
        assert np.any((np.abs(sup_x - px) <= 0.5) & (np.abs(sup_y - py) <= 0.5))
    dmin = min(math.dist(a, b) for i, a in enumerate(pts) for b in pts[i + 1:])
    assert dmin >= r - 1e-12
    S_ = len(sup_x)
    assert r <= math.sqrt(S_ / (12 * math.pi)) + 1e-12
    assert abs(first[:, 2].sum() - 1.0) < 1e-14 and np.all(first[:, 2] > 0)
    rest = S.split_layers(th, taps)[1:]
    radii = [float(np.hypot(l[0, 0], l[0, 1])) for l in rest]
    assert abs(sum(radii) - r) < 1e-12


def test_random_init_bounds():
    K = gaussian_kernel(31, 5.0)
    taps = [8, 8, 8]
    th = I.random_init(K, taps, seed=1)
    dr = 2 * I.radial_extent(K) / 12
    for l, lay in enumerate(S.split_layers(th, taps)):
        assert np.all(np.abs(lay[:, :2]) <= (l + 1) * dr)
        assert abs(lay[:, 2].sum() - 1) < 1e-15


def test_interp_nodes_exact_linear_and_convex():
    G = 9
    basis = np.random.default_rng(5).standard_normal((G, 10, 3))
    for k in range(G):
        P = np.full((1, 2, 3), k / (G - 1))        # exact binary fractions
        for tap in range(10):
            ox, oy, w = IP.tap_field(basis, P, [G], tap)
            assert np.all(ox == basis[k, tap, 0]) and np.all(w == basis[k, tap, 2])
    P = np.linspace(0, 1, 101)
    a = IP.alpha_1d(P, G)
    assert np.allclose(a.sum(-1), 1.0, atol=1e-15) and np.all(a >= 0)
    # linear between nodes: value at the midpoint is the mean of the two nodes
    mid = np.full((1, 1, 1), 2.5 / (G - 1))
    ox, _, _ = IP.tap_field(basis, mid, [G], 4)
    assert abs(ox[0, 0] - 0.5 * (basis[2, 4, 0] + basis[3, 4, 0])) < 1e-15
    # clamping outside [0, 1]
    lo = IP.tap_field(basis, np.full((1, 1, 1), -0.3), [G], 1)[2]
    hi = IP.tap_field(basis, np.full((1, 1, 1), 1.7), [G], 1)[2]
    assert lo[0, 0] == basis[0, 1, 2] and hi[0, 0] == basis[-1, 1, 2]
    # a constant basis gives a P-independent filter
    cb = np.repeat(basis[:1], G, axis=0)
    Pr = np.random.default_rng(1).random((1, 4, 4))
    assert np.allclose(IP.tap_field(cb, Pr, [G], 3)[0], basis[0, 3, 0], atol=1e-15)
    # dense alpha combination equals the per-tap form
    Pr1 = Pr[0]
    full = IP.combine(basis, IP.alpha_1d(Pr1, G))
    ox, oy, w = IP.tap_field(basis, Pr, [G], 6)
    np.testing.assert_allclose(full[..., 6, 0], ox, atol=1e-14)


def test_interp_2d_nodes_and_convexity():
    G0, G1 = 5, 3
    basis = np.random.default_rng(6).standard_normal((G0 * G1, 4, 3))
    for i0 in range(G0):
        for i1 in range(G1):
            P = np.zeros((2, 1, 1))
            P[0] = i0 / (G0 - 1)
            P[1] = i1 / (G1 - 1)
            v = IP.tap_field(basis, P, [G0, G1], 2)
            assert [float(c[0, 0]) for c in v] == list(basis[i0 * G1 + i1, 2])
    P0, P1 = np.random.default_rng(2).random((2, 7))
    a = IP.alpha_2d(P0, P1, G0, G1)
    assert np.allclose(a.sum(-1), 1.0, atol=1e-15) and np.all(a >= 0)


def _basis(G, taps, seed):
    rows = [random_theta(taps, 2.0 + 1.5 * k, seed=seed + k).astype(np.float64) for k in range(G)]
    b = np.stack(rows)
    t0 = 0
    for n in taps:                                # unit weight sum per layer and entry
        b[:, t0:t0 + n, 2] /= b[:, t0:t0 + n, 2].sum(axis=1, keepdims=True)
        t0 += n
    return b


def test_sv_constant_map_is_uniform_chain():
    taps = [5, 4, 6]
    G = 6
    basis = _basis(G, taps, 40)
    img = noise_image(24, 31, 3, seed=2, n_rects=10).astype(np.float64)
    P = np.full((1, 24, 31), 0.37)
    theta = IP.combine(basis, IP.alpha_1d(np.array(0.37), G))
    np.testing.assert_allclose(SV.sv_chain(img, P, basis, [G], taps),
                               S.chain(img, theta, taps, S.CLAMP), rtol=0, atol=1e-13)
    # at a node the result is the uniform chain with that entry
    Pn = np.full((1, 24, 31), 3 / (G - 1))
    k = int(round(float(Pn[0, 0, 0]) * (G - 1)))
    got = SV.sv_chain(img, Pn, basis, [G], taps)
    np.testing.assert_allclose(got, S.chain(img, basis[k], taps, S.CLAMP), rtol=0, atol=1e-13)


def test_sv_single_pass_uses_each_pixels_own_filter():
    taps = [7]
    G = 5
    basis = _basis(G, taps, 50)
    img = noise_image(20, 26, 2, seed=3, n_rects=8).astype(np.float64)
    P = param_map(20, 26, seed=4, period=16.0)
    out = SV.sv_chain(img, P, basis, [G], taps)
    for (y, x) in [(0, 0), (5, 17), (19, 25), (11, 3), (7, 22)]:
        theta = IP.combine(basis, IP.alpha_1d(np.array(float(P[0, y, x])), G))
        want = S.chain(img, theta, taps, S.CLAMP)[:, y, x]
        np.testing.assert_allclose(out[:, y, x], want, rtol=0, atol=1e-14)


def test_sv_constant_image_stays_constant_with_unit_layer_sums():
    taps = [6, 6]
    basis = _basis(4, taps, 60)
    P = param_map(16, 16, seed=9, period=8.0)
    img = np.full((1, 16, 16), 0.625)
    np.testing.assert_allclose(SV.sv_chain(img, P, basis, [4], taps), 0.625, rtol=1e-14)


def test_rotate_basis_quarter_turn_rotates_the_response():
    """Rotating every offset by +90 degrees rotates the chain's impulse
    response by a quarter turn (bilinear reads commute with 90-degree grid
    rotations); angle 0 is the identity and rotations compose."""
    from oracle import interp as IP
    from oracle import sparse as S
    from synth import random_theta
    taps = [5, 4]
    th = random_theta(taps, 3.0, seed=41).astype(np.float64)
    r = IP.rotate_basis(th[None], [0.0, np.pi / 2, np.pi / 3, np.pi / 6])
    np.testing.assert_array_equal(r[0], th)
    K = S.impulse_response(17, th, taps)
    Kq = S.impulse_response(17, r[1], taps)
    np.testing.assert_allclose(Kq, np.rot90(K, k=-1), atol=1e-15)
    twice = IP.rotate_basis(r[3][None], [np.pi / 6])[0]
    np.testing.assert_allclose(twice, r[2], atol=1e-13)


def test_ss_init_layer1_weights_follow_the_target_at_the_rounded_points():
    """Eq. 7's first layer: each tap's weight is the target value at the pixel
    nearest to its sample point, normalised to unit sum.  The target's values
    are all distinct (a ramp over the support), so equal weights, a wrong
    rounding or a transposed lookup all change them."""
    M = 41
    c = (M - 1) // 2
    y, x = np.mgrid[0:M, 0:M]
    K = np.where(np.hypot(x - c, y - c) <= 15.0, 1.0 + 0.37 * x + 0.011 * y * y, 0.0)
    taps = [10, 8, 8]
    th, _ = I.ss_init(K, taps, seed=12, index=5)
    first = th[:10]
    rx = np.floor(first[:, 0] + c + 0.5).astype(int)
    ry = np.floor(first[:, 1] + c + 0.5).astype(int)
    want = K[ry, rx] / K[ry, rx].sum()
    assert np.ptp(want) > 0.05                       # the weights really differ
    np.testing.assert_allclose(first[:, 2], want, rtol=1e-14, atol=0)
