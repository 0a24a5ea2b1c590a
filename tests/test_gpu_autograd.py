"""The hand-written adjoint behind torch.autograd.Function (the filter as a
trainable layer, Sec. 6), checked by central finite differences of the GPU
forward (h = 1e-4, 64 seeded coordinates) and against the FP64 oracle's
gradient, on the differentiation configuration: a 63 x 63 non-convex target,
4 layers x 12 taps, shape-aware init."""
import numpy as np
import pytest
import torch

import paper_2512_04556_amd as disk
from paper_2512_04556_amd.autograd import DiskChain
from oracle import adjoint as A
from oracle import loss as Lo
from synth import shape_batch, uniform_image, random_theta
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _loss_fn(theta, target, taps, M):
    K = DiskChain.apply(theta, None, taps, disk.ZERO, M, M)[0]
    pk = target.max()
    return torch.mean((K - target) ** 2) / (pk * pk)


def test_impulse_autograd_fd_and_oracle(dev):
    M, taps = 63, [12, 12, 12, 12]
    K = shape_batch(1, M, 4, 12, seed=4).kernels[0]
    th0, _ = disk.disk_init_shape(K, taps, seed=4, index=0)
    theta = th0.cuda().requires_grad_(True)
    tgt = torch.as_tensor(K).cuda()
    say("autograd impulse", M, taps)
    loss = _loss_fn(theta, tgt, taps, M)
    loss.backward()
    g = theta.grad.detach().cpu().numpy().astype(np.float64)
    # oracle gradient of the same loss at the same FP32 parameters
    _, _, go = A.impulse_loss_grad(K.astype(np.float64), th0.numpy().astype(np.float64), taps, Lo.NMSE)
    e_or = np.abs(g - go).max() / np.abs(go).max()
    # central differences of the FP64 oracle's loss (h = 1e-4), criterion
    # |g - fd| <= 1e-3 max(|fd|, 1e-3 max|fd|); the same differences of the GPU
    # FP32 forward are reported only (FP32 loss rounding dominates them)
    # Offsets within 10h of an integer sit on a kink of the bilinear read (its
    # derivative is one-sided there), so such coordinates are redrawn.
    rng = np.random.default_rng(64)
    h = 1e-4
    th64 = th0.numpy().astype(np.float64)
    idx = []
    while len(idx) < 64:
        r, c = int(rng.integers(0, th0.shape[0])), int(rng.integers(0, 3))
        f = th64[r, c] - np.floor(th64[r, c])
        if c < 2 and (f < 10 * h or f > 1 - 10 * h):
            continue
        idx.append((r, c))
    fds, gpu_fd = [], []
    for (r, c) in idx:
        tp = th64.copy(); tp[r, c] += h
        tm = th64.copy(); tm[r, c] -= h
        lp = A.impulse_loss_grad(K.astype(np.float64), tp, taps)[0]
        lm = A.impulse_loss_grad(K.astype(np.float64), tm, taps)[0]
        fds.append((lp - lm) / (2 * h))
        tpg = th0.clone(); tpg[r, c] += h
        tmg = th0.clone(); tmg[r, c] -= h
        with torch.no_grad():
            gpu_fd.append((float(_loss_fn(tpg.cuda(), tgt, taps, M)) - float(_loss_fn(tmg.cuda(), tgt, taps, M))) / (2 * h))
    fds = np.array(fds)
    scale = 1e-3 * np.abs(fds).max()
    worst = max(abs(g[r, c] - f) / max(abs(f), scale) for (r, c), f in zip(idx, fds))
    worst_gpu = max(abs(g[r, c] - f) / max(abs(f), scale) for (r, c), f in zip(idx, gpu_fd))
    print(f"FD on the GPU FP32 forward (reported): worst rel err {worst_gpu:.2e}")
    print(f"autograd: vs oracle {e_or:.2e}, worst FD rel err {worst:.2e}")
    assert e_or <= 1e-5
    assert worst <= 1e-3


def test_image_autograd_gradients(dev):
    """Image mode, CLAMP: gradients w.r.t. Theta and the input against the oracle."""
    taps = [6, 5]
    th = random_theta(taps, 4.0, seed=12)
    img = uniform_image(40, 50, 3, seed=3)
    G = np.random.default_rng(2).standard_normal((3, 40, 50)).astype(np.float32)
    theta = torch.as_tensor(th).cuda().requires_grad_(True)
    x = torch.as_tensor(img).cuda().requires_grad_(True)
    say("autograd image")
    y = DiskChain.apply(theta, x, taps, disk.CLAMP)
    (y * torch.as_tensor(G).cuda()).sum().backward()
    wt, wi = A.chain_vjp(img.astype(np.float64), th.astype(np.float64), taps, 1, G.astype(np.float64))
    et = np.abs(theta.grad.cpu().numpy() - wt).max() / np.abs(wt).max()
    ei = np.abs(x.grad.cpu().numpy() - wi).max() / np.abs(wi).max()
    print(f"image autograd: dtheta {et:.2e} dinput {ei:.2e}")
    assert et <= 1e-5 and ei <= 1e-5


def test_image_autograd_bf16_input(dev):
    """A BF16 image: the forward reads BF16 and writes BF16; the adjoint reads
    the image widened to FP32 (exact), so dTheta and dX equal the oracle's on
    the BF16-rounded image and the BF16 output gradient; dX comes back in
    BF16."""
    from tests.gpu_util import bf16_round, rel_err, TOL_F32
    taps = [6, 5, 4]
    th = random_theta(taps, 3.0, seed=14)
    img = uniform_image(37, 70, 3, seed=8)
    G = np.random.default_rng(6).standard_normal((3, 37, 70)).astype(np.float32)
    theta = torch.as_tensor(th).cuda().requires_grad_(True)
    x = torch.as_tensor(img).cuda().bfloat16().requires_grad_(True)
    say("autograd image bf16")
    y = DiskChain.apply(theta, x, taps, disk.CLAMP)
    assert y.dtype == torch.bfloat16
    (y.float() * torch.as_tensor(G).cuda()).sum().backward()
    assert x.grad.dtype == torch.bfloat16
    # autograd hands the chain the gradient of its BF16 output in BF16, so the
    # adjoint's G_L is G rounded to BF16
    wt, wi = A.chain_vjp(bf16_round(img), th.astype(np.float64), taps, 1, bf16_round(G))
    et = rel_err(theta.grad.cpu().numpy(), wt)
    ei = rel_err(x.grad.float().cpu().numpy(), bf16_round(wi))
    print(f"image autograd bf16: dtheta {et:.2e} dinput (BF16 output) {ei:.2e}")
    assert et <= TOL_F32 and ei <= 5e-3


def test_backward_refuses_non_fp32_operands(dev):
    """The C adjoint reads the input, the saved intermediates, the output
    gradient and Theta as FP32: the binding refuses anything else before a
    launch."""
    taps = [4, 4]
    th = torch.as_tensor(random_theta(taps, 2.0, seed=3)).cuda()
    x = torch.as_tensor(uniform_image(16, 16, 3, seed=1)).cuda()
    out, saved = disk.disk_forward(th, taps, x, save=True)
    g = torch.ones_like(out)
    for args in ((th, taps, x.bfloat16(), saved, g), (th, taps, x, saved.bfloat16(), g),
                 (th, taps, x, saved, g.bfloat16()), (th.double(), taps, x, saved, g),
                 (th, taps, x[:, :8], saved, g), (th, taps, x, saved[:, :, :8], g)):
        with pytest.raises(disk.DiskError):
            disk.disk_backward(*args)
