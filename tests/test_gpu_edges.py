"""Edge cases and maximum sizes through the C ABI against the FP64 oracle:
the largest layer structure (8 layers x 32 taps, T = 256) on impulse
canvases up to the maximum side 255 and on ragged 4-channel images, a 1 x 1
image and a 1 x 1 target, and the optimiser on a maximum-side,
maximum-structure target."""
import numpy as np
import pytest
import torch

import paper_2512_04556_amd as disk
from oracle import adam as Ad
from oracle import adjoint as A
from oracle import init as I
from oracle import sparse as S
from oracle import svfilter as SV
from synth import TargetBatch, disk_kernel, noise_image, random_theta
from tests.gpu_util import say, to_dev, to_np, rel_err, bf16_round, TOL_F32, TOL_BF16

pytestmark = pytest.mark.gpu

TAPS_MAX = [32] * 8


def test_max_structure_impulse_forward_and_adjoint(dev):
    """8 layers x 32 taps on the largest impulse canvas (255 x 255, ZERO)."""
    th = random_theta(TAPS_MAX, 6.0, seed=255)
    M = 255
    G = np.random.default_rng(5).standard_normal((1, M, M)).astype(np.float32)
    say("max structure impulse", M)
    out, saved = disk.disk_forward(to_dev(th), TAPS_MAX, None, H=M, W=M, save=True)
    want = S.impulse_response(M, th.astype(np.float64), TAPS_MAX)
    e1 = rel_err(to_np(out), want)
    gt, _ = disk.disk_backward(to_dev(th), TAPS_MAX, None, saved, to_dev(G), need_input=False)
    wt, _ = A.chain_vjp(S.impulse(M)[None], th.astype(np.float64), TAPS_MAX, S.ZERO, G.astype(np.float64))
    e2 = rel_err(to_np(gt), wt)
    print(f"8 x 32 taps on 255 x 255: forward {e1:.2e}, dTheta {e2:.2e}")
    assert e1 <= TOL_F32 and e2 <= TOL_F32


@pytest.mark.parametrize("C,H,W", [(4, 37, 70), (3, 1, 1), (4, 2, 65)])
def test_max_structure_image_chain(dev, C, H, W):
    """8 layers x 32 taps on ragged images (tile tails in both directions),
    a 1 x 1 image and a 2-row image, CLAMP: forward, dTheta and dX."""
    th = random_theta(TAPS_MAX, 3.0, seed=H * W + C)
    img = noise_image(H, W, C, seed=C + H, n_rects=3) if H > 1 else np.random.default_rng(3).random(
        (C, H, W)).astype(np.float32)
    G = np.random.default_rng(H + W).standard_normal((C, H, W)).astype(np.float32)
    say("max structure image chain", C, H, W)
    out, saved = disk.disk_forward(to_dev(th), TAPS_MAX, to_dev(img), boundary=S.CLAMP, save=True)
    want = S.chain(img.astype(np.float64), th.astype(np.float64), TAPS_MAX, S.CLAMP)
    gt, gi = disk.disk_backward(to_dev(th), TAPS_MAX, to_dev(img), saved, to_dev(G), boundary=S.CLAMP)
    wt, wi = A.chain_vjp(img.astype(np.float64), th.astype(np.float64), TAPS_MAX, S.CLAMP, G.astype(np.float64))
    e = (rel_err(to_np(out), want), rel_err(to_np(gt), wt), rel_err(to_np(gi), wi))
    print(f"8 x 32 taps, {C} x {H} x {W}: forward {e[0]:.2e} dTheta {e[1]:.2e} dX {e[2]:.2e}")
    assert max(e) <= TOL_F32


@pytest.mark.parametrize("C,grid,io", [(3, [16], torch.float32), (4, [4, 4], torch.float32),
                                      (3, [16], torch.bfloat16)])
def test_sv_filter_max_structure(dev, C, grid, io):
    """The spatially varying filter with the largest layer structure (8 layers
    x 32 taps, T = 256: the layer tables no longer fit the LDS beside the
    tile) on a ragged multi-tile image, 1-D and 2-D bases, against the
    oracle on the whole image."""
    G = int(np.prod(grid))
    basis = np.stack([random_theta(TAPS_MAX, 1.0 + 0.25 * k, seed=70 + k) for k in range(G)]).astype(np.float32)
    H, W = 45, 140
    img = noise_image(H, W, C, seed=C + 50, n_rects=6)
    rng = np.random.default_rng(C + 60)
    P = rng.random((len(grid), H, W)).astype(np.float32)
    b = disk.make_basis(to_dev(basis), TAPS_MAX, grid)
    say("sv filter max structure", C, grid, io, b.halo)
    out = disk.disk_sv_filter(b, to_dev(img).to(io), to_dev(P))
    x = img.astype(np.float64) if io == torch.float32 else bf16_round(img)
    want = SV.sv_chain(x, P.astype(np.float64), basis.astype(np.float64), grid, TAPS_MAX)
    e = rel_err(to_np(out), want)
    print(f"sv 8 x 32 taps C={C} grid={grid} {io} halo={b.halo}: {e:.2e}")
    assert e <= (TOL_F32 if io == torch.float32 else TOL_BF16)


@pytest.mark.parametrize("H,W,r0,want_max", [(1, 1, 26.5, 30), (2, 65, 26.5, 30), (1, 1, 39.0, 41), (3, 70, 39.0, 41)])
def test_sv_filter_tiny_images_large_halo(dev, H, W, r0, want_max):
    """Images far smaller than the halo on the large-halo paths (the wide
    staged C = 3 kernel at halos up to 30, plane groups up to 41): every
    staged read clamps into the few pixels; against the oracle."""
    taps = [6, 6, 5]
    basis = np.stack([random_theta(taps, r0 + 0.3 * k, seed=(720 if r0 < 30 else 820) + k)
                      for k in range(9)]).astype(np.float32)
    img = np.random.default_rng(H * W).random((3, H, W)).astype(np.float32)
    P = np.random.default_rng(H + W).random((2, H, W)).astype(np.float32)
    b = disk.make_basis(to_dev(basis), taps, [3, 3])
    assert max(b.halo) == want_max
    say("sv tiny image large halo", H, W, b.halo)
    out = disk.disk_sv_filter(b, to_dev(img), to_dev(P))
    want = SV.sv_chain(img.astype(np.float64), P.astype(np.float64), basis.astype(np.float64), [3, 3], taps)
    e = rel_err(to_np(out), want)
    print(f"sv {H} x {W} halo={b.halo}: {e:.2e}")
    assert e <= TOL_F32


def test_sv_filter_one_pixel_image(dev):
    """The SV filter on a 1 x 1 x 3 image: every read clamps to the one pixel,
    so the output is the pixel times the product of the layers' weight sums
    at its own Theta; against the oracle."""
    taps = [8, 8, 8, 8]
    basis = np.stack([random_theta(taps, 1.0 + k, seed=40 + k) for k in range(4)]).astype(np.float32)
    img = np.array([[[0.25]], [[0.5]], [[0.75]]], np.float32)
    P = np.array([[[0.37]]], np.float32)
    b = disk.make_basis(to_dev(basis), taps, [4])
    say("sv filter 1 x 1")
    out = disk.disk_sv_filter(b, to_dev(img), to_dev(P))
    want = SV.sv_chain(img.astype(np.float64), P.astype(np.float64), basis.astype(np.float64), [4], taps)
    assert rel_err(to_np(out), want) <= TOL_F32


def _one(K, taps):
    return TargetBatch([K.astype(np.float32)], np.array([len(taps)], np.int32), [np.array(taps, np.int32)], [{}])


@pytest.mark.parametrize("M,taps", [(255, TAPS_MAX), (1, [3, 2])])
def test_optimizer_extreme_targets_one_step(dev, M, taps):
    """One Adam step on the largest target (side 255, 8 x 32 taps, radial
    init) and on a 1 x 1 target, against the oracle: components whose
    gradient is above 1e-3 of the largest move by exactly lr (1e-6)."""
    from synth import pack_targets
    K = disk_kernel(100.0, M) if M > 1 else np.ones((1, 1), np.float32)
    batch = _one(K, taps)
    th0 = I.radial_init(K.astype(np.float64), taps).astype(np.float32)
    if M == 1:
        th0[:, :2] = np.random.default_rng(2).uniform(-0.4, 0.4, (th0.shape[0], 2))
    bt = disk.make_batch(*pack_targets(batch))
    th = torch.as_tensor(th0).cuda().contiguous()
    say("optimizer extreme target", M, len(taps))
    ps, st, stat = disk.disk_optimize_batch(bt, th, disk.OptParams(max_steps=1, lr0=1e-2, lr1=1e-2))
    _, _, g = A.impulse_loss_grad(K.astype(np.float64), th0.astype(np.float64), taps)
    want, _, _ = Ad.adam_update(th0.astype(np.float64), g, np.zeros_like(g), np.zeros_like(g), 1, 1e-2)
    got = th.cpu().numpy().astype(np.float64)
    assert int(st[0]) == 1 and int(stat[0]) == 0
    big = np.abs(g) > 1e-3 * np.abs(g).max()
    print(f"side {M}, {len(taps)} x {taps[0]} taps: {int(big.sum())} of {g.size} components well determined")
    np.testing.assert_allclose(got[big], want[big], rtol=0, atol=1e-6)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-2 + 1e-6)
