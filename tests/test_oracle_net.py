"""Pins of the learned initialiser's oracle (oracle/net.py) against library
routines (torch conv2d / linear / autograd / bfloat16 casts / Adam, all on
the CPU in float64), finite differences and exact area integration."""
import numpy as np
import pytest
import torch

from oracle import net as N


def test_param_count_and_layout():
    assert N.param_count() == 1_330_960
    shapes = N.param_shapes()
    assert shapes[0] == ((32, 1, 3, 3), (32,))
    assert shapes[5] == ((256, 256, 3, 3), (256,))
    assert shapes[-1] == ((144, 512), (144,))


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = rng.standard_normal(20000) * np.exp(rng.uniform(-20, 20, 20000))
    # exact ties in FP32: low 16 bits = 0x8000, both parities of bit 16
    exp = rng.integers(100, 150, 2000).astype(np.uint32) << np.uint32(23)
    mant = rng.integers(0, 64, 2000).astype(np.uint32) << np.uint32(17)      # bit 16 clear: ties to even
    sign = rng.integers(0, 2, 2000).astype(np.uint32) << np.uint32(31)
    ties = sign | exp | mant | np.uint32(0x8000)
    ties2 = ties | np.uint32(0x10000)                                        # bit 16 set: ties to odd
    x = np.concatenate([x, ties.view(np.float32), ties2.view(np.float32), [0.0, -0.0, 1.0, 65504.0]])
    want = torch.tensor(x, dtype=torch.float64).to(torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(N.to_bf16(x), want)


def _torch_model(flat, layers, round_bf16):
    pairs = [(torch.tensor(W), torch.tensor(b)) for W, b in N.unflatten(flat, layers)]

    def rb(t):
        return t.to(torch.float32).to(torch.bfloat16).to(torch.float64) if round_bf16 else t

    def f(x, params=None):
        a = rb(x[:, None] if x.dim() == 3 else x)
        for li, ((kind, _, _), (W, b)) in enumerate(zip(layers, params or pairs)):
            Wq = rb(W)
            if kind == "conv":
                z = torch.nn.functional.conv2d(a, Wq, b, stride=2, padding=1)
            else:
                z = torch.nn.functional.linear(a.reshape(a.shape[0], -1), Wq, b)
            if li == len(layers) - 1:
                return z
            a = rb(torch.relu(z))
    return f, pairs


@pytest.mark.parametrize("exact", [True, False])
def test_forward_matches_torch(exact):
    lays = N.arch()
    flat = N.init_params(1)
    flat = flat + 0.01 * np.random.default_rng(2).standard_normal(flat.shape)   # non-zero biases
    x = np.random.default_rng(3).uniform(0, 1, (2, 64, 64))
    y, _ = N.forward(flat, x, exact=exact)
    f, _ = _torch_model(flat, lays, not exact)
    want = f(torch.tensor(x)).numpy()
    err = np.abs(y - want).max() / np.abs(want).max()
    assert err < 1e-12, err


def test_backward_exact_matches_torch_autograd():
    lays = N.arch()
    flat = N.init_params(4) + 0.01 * np.random.default_rng(5).standard_normal(N.param_count())
    x = np.random.default_rng(6).uniform(0, 1, (3, 64, 64))
    y = np.random.default_rng(7).standard_normal((3, 144)) * 0.1
    yh, cache = N.forward(flat, x, exact=True)
    g = N.backward(flat, cache, yh, y, exact=True)
    f, pairs = _torch_model(flat, lays, False)
    for W, b in pairs:
        W.requires_grad_(True)
        b.requires_grad_(True)
    out = f(torch.tensor(x), pairs)
    loss = torch.mean((out - torch.tensor(y)) ** 2)
    loss.backward()
    want = np.concatenate([np.concatenate([W.grad.numpy().reshape(-1), b.grad.numpy()]) for W, b in pairs])
    assert abs(N.loss(yh, y) - loss.item()) < 1e-14
    err = np.abs(g - want).max() / np.abs(want).max()
    assert err < 1e-10, err


def test_backward_toy_net_finite_differences():
    """Two layers (conv 1->2 on 8 x 8, FC 32->3), every parameter, h = 1e-6."""
    lays = [("conv", 1, 2), ("fc", 32, 3)]
    flat = N.init_params(8, lays) + 0.1 * np.random.default_rng(9).standard_normal(N.param_count(lays))
    x = np.random.default_rng(10).uniform(-1, 1, (2, 8, 8))
    y = np.random.default_rng(11).standard_normal((2, 3))
    yh, cache = N.forward(flat, x, lays, exact=True)
    g = N.backward(flat, cache, yh, y, exact=True)
    h = 1e-6
    fd = np.zeros_like(flat)
    for i in range(flat.size):
        fp = flat.copy(); fp[i] += h
        fm = flat.copy(); fm[i] -= h
        fd[i] = (N.loss(N.forward(fp, x, lays, exact=True)[0], y) - N.loss(N.forward(fm, x, lays, exact=True)[0], y)) / (2 * h)
    err = np.abs(g - fd).max() / np.abs(fd).max()
    assert err < 1e-7, err


class _RoundFwd(torch.autograd.Function):
    """Forward: round to FP32 then BF16; backward: identity."""
    @staticmethod
    def forward(ctx, t):
        return t.to(torch.float32).to(torch.bfloat16).to(torch.float64)

    @staticmethod
    def backward(ctx, g):
        return g


class _RoundGrad(torch.autograd.Function):
    """Forward: identity; backward: round the incoming gradient (FP32, or
    FP32 then BF16)."""
    @staticmethod
    def forward(ctx, t, bf16):
        ctx.bf16 = bf16
        return t.view_as(t)

    @staticmethod
    def backward(ctx, g):
        g = g.to(torch.float32)
        if ctx.bf16:
            g = g.to(torch.bfloat16)
        return g.to(torch.float64), None


def test_rounded_backward_matches_torch_autograd_with_rounding_nodes():
    """The BF16 model's backward against torch autograd of the same model with
    the rounding placed as autograd nodes: the bias sees dL/dz in FP32, both
    contractions see it in BF16, weights and activations are rounded in the
    forward pass only."""
    lays = N.arch()
    flat = N.init_params(12) + 0.01 * np.random.default_rng(13).standard_normal(N.param_count())
    x = N.to_bf16(np.random.default_rng(14).uniform(0, 1, (2, 64, 64)))
    y = np.random.default_rng(15).standard_normal((2, 144)) * 0.1
    yr, cr = N.forward(flat, x)
    gr = N.backward(flat, cr, yr, y)
    pairs = [(torch.tensor(W, requires_grad=True), torch.tensor(b, requires_grad=True))
             for W, b in N.unflatten(flat, lays)]
    a = torch.tensor(x)[:, None]
    for li, ((kind, _, _), (W, b)) in enumerate(zip(lays, pairs)):
        Wq = _RoundFwd.apply(W)
        if kind == "conv":
            c = torch.nn.functional.conv2d(a, Wq, None, stride=2, padding=1)
            z = _RoundGrad.apply(_RoundGrad.apply(c, True) + b[None, :, None, None], False)
        else:
            c = a.reshape(a.shape[0], -1) @ Wq.T
            z = _RoundGrad.apply(_RoundGrad.apply(c, True) + b, False)
        a = z if li == len(lays) - 1 else _RoundFwd.apply(torch.relu(z))
    loss = torch.mean((a - torch.tensor(y)) ** 2)
    loss.backward()
    want = np.concatenate([np.concatenate([W.grad.numpy().reshape(-1), b.grad.numpy()]) for W, b in pairs])
    np.testing.assert_allclose(a.detach().numpy(), yr, rtol=0, atol=1e-13)
    err = np.abs(gr - want).max() / np.abs(want).max()
    assert err < 1e-10, err


def test_adam_matches_torch():
    rng = np.random.default_rng(16)
    p0 = rng.standard_normal(50)
    p = torch.nn.Parameter(torch.tensor(p0.copy()))
    opt = torch.optim.Adam([p], lr=3e-4)
    th, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for s in range(1, 6):
        g = rng.standard_normal(50)
        p.grad = torch.tensor(g)
        opt.step()
        th, m, v = N.adam(th, g, m, v, s, 3e-4)
    np.testing.assert_allclose(th, p.detach().numpy(), rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("M", [15, 63, 65, 127])
def test_area_resampling_exact_integration(M):
    """Brute force: split every target pixel into 64 x 64 sub-pixels and bin
    them into the cells; every cell edge falls on a sub-pixel edge, so this
    is the exact area average.  Also: mass is preserved (sum x s^2 = sum K)."""
    rng = np.random.default_rng(M)
    K = rng.uniform(0, 1, (M, M))
    A, s = N.area_matrix(M)
    n = 64
    sub = (np.arange(M * n) + 0.5) / n - 0.5          # sub-pixel centres in target coordinates
    c = (M - 1) / 2
    cell = np.floor((sub - c) / s + 32).astype(int)
    B = np.zeros((64, M))
    ok = (cell >= 0) & (cell < 64)
    np.add.at(B, (cell[ok], np.repeat(np.arange(M), n)[ok]), 1.0 / (n * s))
    np.testing.assert_allclose(A, B, atol=1e-12)
    x = A @ K @ A.T
    assert abs(x.sum() * s * s - K.sum()) < 1e-9 * K.sum()


def test_prepare_input_symmetry_and_peak():
    from synth import gaussian_kernel
    x, hw = N.prepare_input(gaussian_kernel(31, 4.0), exact=True)
    assert hw == 32.0
    assert abs(x.max() - 1.0) < 1e-15
    np.testing.assert_allclose(x, x[::-1, ::-1], atol=1e-15)
    x2, hw2 = N.prepare_input(gaussian_kernel(127, 10.0))
    assert hw2 == 63.5
    np.testing.assert_array_equal(x2, N.to_bf16(x2))
