"""GPU parity of the spatially varying filter (Sec. 4.3, Eq. 8-9) against the
FP64 oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import paper_2512_04556_amd as disk
from oracle import svfilter as SV
from oracle import sparse as S
from synth import random_theta, noise_image, param_map
from tests.gpu_util import say, to_dev, to_np, bf16_round, rel_err, TOL_F32, TOL_BF16

pytestmark = pytest.mark.gpu


def _basis(G, taps, seed, r0=1.0, dr=1.0):
    """Entries whose offsets grow with k, like a family of blurs."""
    return np.stack([random_theta(taps, r0 + dr * k, seed=seed + k) for k in range(G)]).astype(np.float32)


def _run(basis, taps, grid, img, P, io=torch.float32):
    b = disk.make_basis(to_dev(basis), taps, grid)
    x = to_dev(img).to(io)
    out = disk.disk_sv_filter(b, x, to_dev(P))
    return out, b


@pytest.mark.parametrize("C,H,W,pmode,G,taps", [
    (3, 150, 333, "smooth", 16, [8, 8, 8, 8]),
    (3, 97, 130, "noise", 16, [8, 8, 8, 8]),
    (1, 64, 64, "nodes", 9, [6, 6]),
    (2, 77, 200, "outside", 5, [5, 7, 3]),
    (4, 33, 65, "smooth", 1, [8, 4]),
    (3, 1, 70, "smooth", 4, [4, 4]),
])
def test_sv_1d_parity(dev, C, H, W, pmode, G, taps):
    g = np.random.default_rng(H * W)
    basis = _basis(G, taps, seed=G * 10 + C)
    img = noise_image(H, W, C, seed=H, n_rects=15)
    if pmode == "smooth":
        P = param_map(H, W, seed=W, period=96.0)
    elif pmode == "noise":
        P = g.random((1, H, W)).astype(np.float32)
    elif pmode == "nodes":
        P = (g.integers(0, G, (1, H, W)) / (G - 1)).astype(np.float32)
    else:
        P = g.uniform(-0.5, 1.5, (1, H, W)).astype(np.float32)
    say("sv 1d", C, H, W, pmode, G, taps)
    out, b = _run(basis, taps, [G], img, P)
    want = SV.sv_chain(img.astype(np.float64), P.astype(np.float64), basis.astype(np.float64), [G], taps)
    e = rel_err(to_np(out), want)
    print(f"sv1d C={C} {H}x{W} {pmode} G={G} halo={b.halo}: max-abs/peak {e:.2e}")
    assert e <= TOL_F32


def test_sv_2d_bf16_parity(dev):
    taps = [12, 12, 12, 12]
    G0, G1 = 8, 8
    basis = _basis(G0 * G1, taps, seed=77, r0=1.0, dr=0.15)
    H, W = 90, 211
    img = noise_image(H, W, 3, seed=5, n_rects=10)
    P = param_map(H, W, seed=6, period=80.0, dims=2)
    say("sv 2d bf16", H, W)
    out, _ = _run(basis, taps, [G0, G1], img, P, io=torch.bfloat16)
    assert out.dtype == torch.bfloat16
    want = SV.sv_chain(bf16_round(img), P.astype(np.float64), basis.astype(np.float64), [G0, G1], taps)
    e = rel_err(to_np(out), want)
    print(f"sv2d bf16: {e:.2e}")
    assert e <= TOL_BF16


def test_sv_2d_f32_parity_noise_map(dev):
    taps = [6, 6]
    basis = _basis(12, taps, seed=3, dr=0.5)
    H, W = 40, 90
    img = noise_image(H, W, 2, seed=8, n_rects=5)
    P = np.random.default_rng(1).random((2, H, W)).astype(np.float32)
    say("sv 2d f32 noise")
    out, _ = _run(basis, taps, [4, 3], img, P)
    want = SV.sv_chain(img.astype(np.float64), P.astype(np.float64), basis.astype(np.float64), [4, 3], taps)
    assert rel_err(to_np(out), want) <= TOL_F32


def test_sv_halo_violation_gives_nan(dev):
    taps = [4, 4]
    basis = _basis(3, taps, seed=1, r0=3.0)
    b = disk.make_basis(to_dev(basis), taps, [3])
    b.desc.halo[1] = 1                      # declared bound below the real offsets
    img = to_dev(noise_image(20, 70, 1, seed=1, n_rects=2))
    P = to_dev(param_map(20, 70, seed=2, period=32.0))
    say("sv halo violation")
    out = disk.disk_sv_filter(b, img, P)
    assert torch.isnan(out).all()


def test_sv_full_1080p_parity(dev):
    """The benchmark's launch configuration: 1920x1080x3 FP32, 16-entry basis of
    4 x 8 taps (offsets up to ~17 px), smooth blur map; whole frame vs oracle."""
    taps = [8, 8, 8, 8]
    basis = _basis(16, taps, seed=100, r0=1.0, dr=1.05)
    H, W = 1080, 1920
    img = noise_image(H, W, 3, seed=2)
    P = param_map(H, W, seed=3)
    say("sv 1080p full frame")
    out, b = _run(basis, taps, [16], img, P)
    got = to_np(out)
    want = SV.sv_chain(img.astype(np.float64), P.astype(np.float64), basis.astype(np.float64), [16], taps)
    e = rel_err(got, want)
    print(f"sv 1080p halo={b.halo}: max-abs/peak {e:.2e}")
    assert e <= TOL_F32
