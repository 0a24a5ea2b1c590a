"""GPU parity of the dense spatially varying convolution (the per-pixel
kernel the sparse filter approximates) against the FP64 oracle
(oracle.dense.dense_sv with the disk / ellipse coverages), through the C ABI."""
import numpy as np
import pytest
import torch

import paper_2512_04556_amd as disk
from oracle import dense as D
from synth import noise_image, param_map, uniform_image
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _rel(got, want):
    return float(np.abs(got - want).max() / np.abs(want).max())


@pytest.mark.parametrize("C,H,W", [(3, 37, 53), (1, 70, 9), (4, 1, 65)])
def test_dense_disk_parity(dev, C, H, W):
    img = uniform_image(H, W, C, seed=C + H)
    P = param_map(H, W, seed=W)
    r0, r1, half = 0.5, 6.0, 7
    say("dense disk", C, H, W)
    got = disk.disk_dense_sv(torch.as_tensor(img).cuda(), torch.as_tensor(P).cuda(), disk.DENSE_DISK, r0, r1, half)
    want = D.dense_sv(img.astype(np.float64), D.disk_coverage(lambda u: r0 + (r1 - r0) * np.clip(u, 0, 1)),
                      P.astype(np.float64), half)
    assert _rel(got.cpu().numpy(), want) <= 1e-5


def test_dense_ellipse_parity(dev):
    H, W = 45, 60
    img = uniform_image(H, W, 3, seed=8)
    P = param_map(H, W, seed=9, dims=2)
    r0, r1, a0, a1, half = 1.0, 5.0, 0.5, 2.0, 9
    say("dense ellipse")
    got = disk.disk_dense_sv(torch.as_tensor(img).cuda(), torch.as_tensor(P).cuda(), disk.DENSE_ELLIPSE, r0, r1, half,
                             a0, a1)
    cov = D.ellipse_coverage(lambda u: r0 + (r1 - r0) * np.clip(u, 0, 1),
                             lambda u: a0 * (a1 / a0) ** np.clip(u, 0, 1))
    want = D.dense_sv(img.astype(np.float64), cov, P.astype(np.float64), half)
    assert _rel(got.cpu().numpy(), want) <= 1e-5


def test_dense_truncated_window_and_bf16(dev):
    """half below the kernel's reach cuts both sides alike; BF16 I/O within
    the BF16 bar."""
    H, W = 30, 41
    img = uniform_image(H, W, 2, seed=3)
    P = param_map(H, W, seed=4)
    cov = D.disk_coverage(lambda u: 2.0 + 8.0 * np.clip(u, 0, 1))
    want = D.dense_sv(img.astype(np.float64), cov, P.astype(np.float64), 4)
    got = disk.disk_dense_sv(torch.as_tensor(img).cuda(), torch.as_tensor(P).cuda(), disk.DENSE_DISK, 2.0, 10.0, 4)
    assert _rel(got.cpu().numpy(), want) <= 1e-5
    xb = torch.as_tensor(img).to(torch.bfloat16).cuda()
    gb = disk.disk_dense_sv(xb, torch.as_tensor(P).cuda(), disk.DENSE_DISK, 2.0, 10.0, 4)
    wantb = D.dense_sv(xb.float().cpu().numpy().astype(np.float64), cov, P.astype(np.float64), 4)
    assert _rel(gb.float().cpu().numpy(), wantb) <= 5e-3


def test_dense_1080p_crops(dev):
    """The benchmark's reference (disks r = 2 + 30 P, half 33) on the full
    frame; two seeded 48 x 48 crops of the output against the oracle, which
    reads the full image."""
    H, W = 1080, 1920
    img = noise_image(H, W, 3, seed=2)
    P = param_map(H, W, seed=3)
    say("dense 1080p")
    got = disk.disk_dense_sv(torch.as_tensor(img).cuda(), torch.as_tensor(P).cuda(), disk.DENSE_DISK, 2.0, 32.0, 33)
    got = got.cpu().numpy()
    cov = D.disk_coverage(lambda u: 2.0 + 30.0 * np.clip(u, 0, 1))
    rng = np.random.default_rng(11)
    for _ in range(2):
        y0, x0 = int(rng.integers(0, H - 48)), int(rng.integers(0, W - 48))
        rows, cols = slice(y0, y0 + 48), slice(x0, x0 + 48)
        want = D.dense_sv(img.astype(np.float64), cov, P.astype(np.float64), 33, rows, cols)
        assert _rel(got[:, rows, cols], want) <= 1e-5, (y0, x0)
