"""Pins of the oracle's adjoint (Sec. 4.1 end-to-end differentiation), losses
(Eq. 11 and the PSNR metric) and Adam (Sec. 5.1)."""
import os

import numpy as np
import pytest
import torch

from oracle import sparse as S
from oracle import adjoint as A
from oracle import loss as Lo
from oracle import adam as Ad
from synth import random_theta, uniform_image, gaussian_kernel

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _away_from_integers(th, h):
    """Resample offsets so no sample position is within 10h of an integer
    (the bilinear read has kinks there)."""
    th = th.copy()
    for j in range(2):
        f = th[:, j] - np.floor(th[:, j])
        bad = (f < 10 * h) | (f > 1 - 10 * h)
        th[bad, j] += 0.5
    return th


def test_loss_hand_values():
    vals = dict(l.split() for l in open(os.path.join(GOLD, "loss_hand.txt")) if l[0] != "#")
    T = np.array([[0, 1, 0], [1, 4, 1], [0, 1, 0]]) / 8.0
    K = np.zeros((3, 3))
    assert abs(Lo.nmse(K, T) - float(vals["nmse"])) < 1e-16
    assert abs(Lo.psnr_db(K, T) - float(vals["psnr"])) < 1e-12
    assert abs(Lo.charbonnier(K, T) - float(vals["charbonnier"])) < 1e-15


@pytest.mark.parametrize("kind", [Lo.NMSE, Lo.CHARBONNIER])
def test_impulse_gradient_matches_central_fd(kind):
    taps = [5, 6, 4]
    M = 21
    target = gaussian_kernel(M, 3.0)
    th = _away_from_integers(random_theta(taps, 4.0, seed=21).astype(np.float64), 1e-6)
    loss, _, g = A.impulse_loss_grad(target, th, taps, kind)
    h = 1e-6
    fd = np.zeros_like(th)
    for idx in np.ndindex(*th.shape):
        tp = th.copy(); tp[idx] += h
        tm = th.copy(); tm[idx] -= h
        lp = A.impulse_loss_grad(target, tp, taps, kind)[0]
        lm = A.impulse_loss_grad(target, tm, taps, kind)[0]
        fd[idx] = (lp - lm) / (2 * h)
    err = np.abs(g - fd).max() / np.abs(fd).max()
    assert err < 1e-7, err


@pytest.mark.parametrize("boundary", [S.ZERO, S.CLAMP])
def test_image_chain_vjp_fd_and_dot_product(boundary):
    taps = [4, 3]
    th = _away_from_integers(random_theta(taps, 3.0, seed=7).astype(np.float64), 1e-6)
    X = uniform_image(11, 13, 2, seed=5).astype(np.float64)
    G = np.random.default_rng(1).standard_normal((2, 11, 13))

    def f(t, x):
        return float(np.sum(G * S.chain(x, t, taps, boundary)))

    dth, dX = A.chain_vjp(X, th, taps, boundary, G)
    h = 1e-6
    for idx in np.ndindex(*th.shape):
        tp = th.copy(); tp[idx] += h
        tm = th.copy(); tm[idx] -= h
        fd = (f(tp, X) - f(tm, X)) / (2 * h)
        assert abs(dth[idx] - fd) <= 1e-7 * max(1.0, abs(fd)), (idx, dth[idx], fd)
    # the input adjoint is the transpose: <A x, y> = <x, A^T y> (chain is linear in x)
    x2 = uniform_image(11, 13, 2, seed=9).astype(np.float64)
    lhs = np.sum(G * S.chain(x2, th, taps, boundary))
    rhs = np.sum(x2 * dX)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_weight_gradient_closed_form_integer_offsets():
    """Single layer, integer offsets: dL/dw_i = <G, X shifted by o_i>."""
    X = uniform_image(9, 12, 1, seed=3)[0].astype(np.float64)
    G = np.random.default_rng(2).standard_normal((9, 12))
    lay = np.array([[2.0, -1.0, 0.3], [-3.0, 2.0, 0.5], [0.0, 0.0, 0.2]])
    dl, _ = A.layer_vjp(X, lay, S.CLAMP, G)
    y, x = np.mgrid[0:9, 0:12]
    for i, (ox, oy, _) in enumerate(lay):
        sh = X[np.clip(y - int(oy), 0, 8), np.clip(x - int(ox), 0, 11)]
        assert abs(dl[i, 2] - np.sum(G * sh)) < 1e-13


def test_adam_first_step_is_signed_lr():
    g = np.array([[1e-9, -3.0, 0.5]])
    th, _, _ = Ad.adam_update(np.zeros((1, 3)), g, np.zeros((1, 3)), np.zeros((1, 3)), 1, 0.01)
    np.testing.assert_allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-15)


def test_adam_matches_torch_optim_adam_fp64():
    """Same gradients fed to torch.optim.Adam (CPU, float64) with the same
    linear learning-rate schedule."""
    rng = np.random.default_rng(4)
    S_ = 25
    gs = rng.standard_normal((S_, 7, 3))
    th = rng.standard_normal((7, 3))
    p = torch.nn.Parameter(torch.tensor(th.copy(), dtype=torch.float64))
    opt = torch.optim.Adam([p], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    for s in range(S_):
        lr = Ad.lr_at(s, S_, 1e-2, 1e-3)
        for grp in opt.param_groups:
            grp["lr"] = lr
        p.grad = torch.tensor(gs[s], dtype=torch.float64)
        opt.step()
        th, m, v = Ad.adam_update(th, gs[s], m, v, s + 1, lr)
    np.testing.assert_allclose(th, p.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_lr_schedule_endpoints():
    assert Ad.lr_at(0, 1000, 1e-3, 1e-4) == 1e-3
    assert abs(Ad.lr_at(999, 1000, 1e-3, 1e-4) - 1e-4) < 1e-19
    assert Ad.lr_at(0, 1, 1e-3, 1e-4) == 1e-3


def test_optimiser_recovers_a_representable_target():
    """Target = F_Theta_true(delta); from a perturbed start the loop gains
    PSNR, and starting exactly at Theta_true stops before any update."""
    taps = [4, 4]
    M = 17
    th_true = random_theta(taps, 3.0, seed=31).astype(np.float64)
    target = S.impulse_response(M, th_true, taps)
    p = Ad.OptParams(max_steps=150, lr0=1e-2, lr1=1e-3, psnr_stop_db=200.0)
    start = th_true + np.random.default_rng(0).normal(0, 0.15, th_true.shape) * [1, 1, 0.1]
    trace = []
    _, ps, steps = Ad.optimize(target, start, taps, p, trace)
    assert steps == 150 and ps > trace[0][1] + 10.0
    _, ps0, steps0 = Ad.optimize(target, th_true, taps, p)
    assert steps0 == 0 and ps0 == float("inf")


def test_kink_side_is_the_same_at_every_pixel():
    """A tap offset o = +1e-16 samples just left of an integer: floor(p - o)
    = p - 1 at every pixel p, so the offset derivative uses the left segment
    everywhere.  On X[y, x] = x^2 with G = 1 that segment's slope is 2x - 1;
    a rounded p - o would flip to the right segment (2x + 1) once ulp(p) > o."""
    W = 64
    X = np.tile((np.arange(W, dtype=np.float64) ** 2)[None, :], (3, 1))
    G = np.zeros_like(X)
    G[1, 1:] = 1.0                          # columns 1..63, one interior row
    lay = np.array([[1e-16, 0.0, 0.5]])
    dl, _ = A.layer_vjp(X, lay, S.CLAMP, G)
    x = np.arange(1, W, dtype=np.float64)
    assert dl[0, 0] == -0.5 * np.sum(2 * x - 1)


def test_continuation_follows_exact_dilations():
    """Targets that are exact dilations of one representable filter, entry k
    = F(Theta_true with offsets x s^k): started at Theta_true, every entry's
    continuation start is already exact, so no entry takes a step."""
    taps = [4, 3]
    th_true = random_theta(taps, 1.5, seed=5).astype(np.float64)
    s = 1.25
    targets = []
    for k in range(4):
        th = th_true.copy()
        th[:, :2] *= s ** k
        targets.append(S.impulse_response(2 * int(np.ceil(3.5 * s ** k)) + 9, th, taps))
    p = Ad.OptParams(max_steps=50, lr0=1e-2, lr1=1e-3, psnr_stop_db=250.0)
    thetas, ps, steps = Ad.fit_continuation(targets, th_true, taps, [1.0] + [s] * 3, p)
    assert list(steps) == [0, 0, 0, 0]
    assert np.all(ps >= 250.0)
    np.testing.assert_allclose(thetas[3][:, :2], th_true[:, :2] * s ** 3, rtol=1e-14)
    # and a wrong-direction scale does need steps
    _, _, steps2 = Ad.fit_continuation(targets, th_true, taps, [1.0] + [1 / s] * 3, p)
    assert steps2[1] > 0


def test_optimize_loop_is_evaluate_then_adam_with_step_indexed_lr():
    """The loop of Sec. 4.4 / Sec. 5.1: evaluate, then one Adam update with
    the learning rate of step s (linear from lr0 at s = 0 to lr1 at s = S-1)
    and bias correction t = s + 1; after S updates one more evaluation.
    Compared with torch.optim.Adam (float64) driven by the oracle's own
    gradients and a schedule written out here; an off-by-one in the lr index,
    the bias-correction step or the final evaluation fails."""
    taps = [5, 4]
    M = 15
    th_true = random_theta(taps, 2.5, seed=41).astype(np.float64)
    target = S.impulse_response(M, th_true, taps)
    start = th_true + np.random.default_rng(3).normal(0, 0.3, th_true.shape) * [1, 1, 0.05]
    S_, lr0, lr1 = 3, 4e-2, 1e-2
    p = Ad.OptParams(max_steps=S_, lr0=lr0, lr1=lr1)
    trace = []
    th, ps, steps = Ad.optimize(target, start, taps, p, trace)
    q = torch.nn.Parameter(torch.tensor(start, dtype=torch.float64))
    opt = torch.optim.Adam([q], lr=lr0, betas=(0.9, 0.999), eps=1e-8)
    for s in range(S_):
        loss, _, g = A.impulse_loss_grad(target, q.detach().numpy(), taps)
        assert loss == trace[s][0]
        for grp in opt.param_groups:
            grp["lr"] = lr0 + (lr1 - lr0) * s / (S_ - 1)
        q.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
    np.testing.assert_allclose(th, q.detach().numpy(), rtol=1e-13, atol=1e-15)
    assert steps == S_ and len(trace) == S_ + 1
    _, ps_end, _ = A.impulse_loss_grad(target, th, taps)
    assert ps == ps_end == trace[-1][1]


def test_optimize_stops_before_the_update_that_would_pass_the_threshold():
    """Stop rule: a threshold between the PSNR after k and after k + 1
    updates stops with exactly k + 1 updates applied and Theta equal to the
    (k + 1)-update iterate of an unstopped run."""
    taps = [4, 4]
    M = 15
    th_true = random_theta(taps, 2.0, seed=43).astype(np.float64)
    target = S.impulse_response(M, th_true, taps)
    start = th_true + np.random.default_rng(5).normal(0, 0.2, th_true.shape) * [1, 1, 0.05]
    full = []
    Ad.optimize(target, start, taps, Ad.OptParams(max_steps=12, lr0=2e-2, lr1=2e-2), full)
    k = int(np.argmax([b[1] > a[1] for a, b in zip(full[4:], full[5:])])) + 4
    thr = 0.5 * (full[k][1] + full[k + 1][1])
    assert max(f[1] for f in full[:k + 1]) < thr
    th_stop, ps, steps = Ad.optimize(target, start, taps, Ad.OptParams(max_steps=12, lr0=2e-2, lr1=2e-2,
                                                                          psnr_stop_db=thr))
    assert steps == k + 1 and ps == full[k + 1][1]
    th_k, _, _ = Ad.optimize(target, start, taps, Ad.OptParams(max_steps=k + 1, lr0=2e-2, lr1=2e-2))
    # the same k + 1 updates (constant lr, so the schedule length does not matter)
    np.testing.assert_array_equal(th_stop, th_k)


def test_optimize_half_width_offset_units_match_torch_param_groups():
    """Offsets' learning rate in units of the half-width (M - 1) / 2, weights
    at the plain rate: equal to torch.optim.Adam (float64) with two parameter
    groups (offsets at lr * (M - 1) / 2, weights at lr) driven by the oracle's
    gradients; a unit applied to the weights, or a wrong half-width, fails."""
    taps = [5, 4]
    M = 21
    th_true = random_theta(taps, 3.0, seed=44).astype(np.float64)
    target = S.impulse_response(M, th_true, taps)
    start = th_true + np.random.default_rng(6).normal(0, 0.3, th_true.shape) * [1, 1, 0.05]
    S_, lr0, lr1 = 4, 3e-3, 1e-3
    th, ps, steps = Ad.optimize(target, start, taps, Ad.OptParams(max_steps=S_, lr0=lr0, lr1=lr1, offset_units=1))
    off = torch.nn.Parameter(torch.tensor(start[:, :2], dtype=torch.float64))
    w = torch.nn.Parameter(torch.tensor(start[:, 2], dtype=torch.float64))
    opt = torch.optim.Adam([{"params": [off]}, {"params": [w]}], lr=lr0, betas=(0.9, 0.999), eps=1e-8)
    for s in range(S_):
        cur = np.concatenate([off.detach().numpy(), w.detach().numpy()[:, None]], axis=1)
        _, _, g = A.impulse_loss_grad(target, cur, taps)
        lr = lr0 + (lr1 - lr0) * s / (S_ - 1)
        opt.param_groups[0]["lr"] = lr * (M - 1) / 2
        opt.param_groups[1]["lr"] = lr
        off.grad = torch.tensor(g[:, :2], dtype=torch.float64)
        w.grad = torch.tensor(g[:, 2], dtype=torch.float64)
        opt.step()
    want = np.concatenate([off.detach().numpy(), w.detach().numpy()[:, None]], axis=1)
    np.testing.assert_allclose(th, want, rtol=1e-13, atol=1e-15)
    # and the offsets did move further than the pixel-unit run's
    th_px, _, _ = Ad.optimize(target, start, taps, Ad.OptParams(max_steps=S_, lr0=lr0, lr1=lr1))
    assert np.abs(th[:, :2] - start[:, :2]).sum() > 5 * np.abs(th_px[:, :2] - start[:, :2]).sum()
