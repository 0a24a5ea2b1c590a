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


@pytest.mark.parametrize("seed,r0,declared", [(720, 26.5, 26), (820, 39.0, 33)])
def test_sv_halo_violation_large_halo_paths(dev, seed, r0, declared):
    """A declared halo below the real offsets on the large-halo paths (the
    wide staged C = 3 kernel at 26; plane groups at 33): every output NaN."""
    taps = [6, 6, 5]
    basis = _basis(9, taps, seed=seed, r0=r0, dr=0.3)
    b = disk.make_basis(to_dev(basis), taps, [3, 3])
    b.desc.halo[1] = declared
    img = to_dev(noise_image(70, 150, 3, seed=seed, n_rects=6))
    P = to_dev(param_map(70, 150, seed=seed + 5, period=48.0, dims=2))
    say("sv halo violation large", declared)
    out = disk.disk_sv_filter(b, img, P)
    assert torch.isnan(out).all()


@pytest.mark.parametrize("C,io,taps,G", [
    (3, torch.float32, [8, 8, 8, 8], 16),
    (4, torch.float32, [5, 9, 3], 7),
    (3, torch.bfloat16, [12, 12, 12, 12], 16),
])
def test_sv_one_shot_equals_prepared_table(dev, C, io, taps, G):
    """disk_sv_filter on a 1-D basis with C >= 3 derives every layer's
    coefficients inside its pass; the result must be bitwise the one of the
    prepared-table path (disk_sv_prepare + disk_sv_apply)."""
    basis = _basis(G, taps, seed=5 * C + G, r0=1.5, dr=0.9)
    H, W = 123, 301
    img = noise_image(H, W, C, seed=C, n_rects=8)
    P = param_map(H, W, seed=4, period=64.0)
    b = disk.make_basis(to_dev(basis), taps, [G])
    x, p = to_dev(img).to(io), to_dev(P)
    say("sv one-shot vs prepared", C, io, taps, G)
    one = disk.disk_sv_filter(b, x, p)
    prep = disk.disk_sv_apply(b, disk.disk_sv_prepare(b), x, p)
    torch.cuda.synchronize()
    assert torch.equal(one, prep)


@pytest.mark.parametrize("bad_layer", [0, 2])
def test_sv_halo_violation_one_shot_gives_nan(dev, bad_layer):
    """The one-shot path checks each layer's offsets in that layer's pass: a
    violation in any layer still leaves the whole output NaN."""
    taps = [6, 6, 6]
    basis = _basis(5, taps, seed=9, r0=2.0)
    b = disk.make_basis(to_dev(basis), taps, [5])
    b.desc.halo[bad_layer] = 1
    img = to_dev(noise_image(40, 90, 3, seed=3, n_rects=4))
    P = to_dev(param_map(40, 90, seed=5, period=32.0))
    say("sv halo violation one-shot", bad_layer)
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


def test_sv_bench_configuration_full_frame(dev):
    """Exactly the benchmark's workload: the fitted 16-disk basis (continuation
    fit from the radial init, 4 x 8 taps; halos span both pass variants),
    1920x1080x3 FP32; the whole frame against the oracle."""
    from synth import disk_kernel
    taps = [8, 8, 8, 8]
    radii = [2.0 * (k + 1) for k in range(16)]
    th, _, _, _ = disk.fit_basis([disk_kernel(r) for r in radii], taps,
                                 [1.0] + [radii[k] / radii[k - 1] for k in range(1, 16)])
    basis = th.cpu().numpy()
    H, W = 1080, 1920
    img = noise_image(H, W, 3, seed=2)
    P = param_map(H, W, seed=3)
    say("sv bench configuration")
    out, b = _run(basis, taps, [16], img, P)
    want = SV.sv_chain(img.astype(np.float64), P.astype(np.float64), basis.astype(np.float64), [16], taps)
    e = rel_err(to_np(out), want)
    print(f"sv bench config halo={b.halo}: max-abs/peak {e:.2e}")
    assert max(b.halo) > 12 and min(b.halo) <= 12
    assert e <= TOL_F32


def test_sv_2d_4k_bf16_sampled(dev):
    """The 2-D workload at full size: 3840x2160x3 BF16 I/O, 8 x 8 basis of
    4 x 12 taps with halos 27..30 (the wide-halo staged kernel), 2-D map.  Two
    seeded interior 32 x 32 output crops, a top-border, a left-border and the
    bottom-right corner crop against the oracle run on the crop plus a margin
    of the summed halos (the margin's own clamping cannot reach the crop)."""
    taps = [12, 12, 12, 12]
    basis = _basis(64, taps, seed=400, r0=4.0, dr=0.4)
    H, W = 2160, 3840
    img = noise_image(H, W, 3, seed=2)
    P = param_map(H, W, seed=3, dims=2)
    say("sv 2d 4k bf16")
    out, b = _run(basis, taps, [8, 8], img, P, io=torch.bfloat16)
    got = to_np(out)
    assert max(b.halo) > 24
    m = int(sum(b.halo))
    xb = bf16_round(img)
    rng = np.random.default_rng(4)
    crops = [(int(rng.integers(m, H - 32 - m)), int(rng.integers(m, W - 32 - m))) for _ in range(2)]
    # the top border, the bottom-right corner and the left border: the CLAMP
    # edge and the ends of the tile runs (the crop's margin is clipped at the
    # image's edge, where the oracle's own CLAMP border is the image's)
    crops += [(0, 1900), (H - 32, W - 32), (1000, 0)]
    for y0, x0 in crops:
        ya, yb, xa, xb_ = max(0, y0 - m), min(H, y0 + 32 + m), max(0, x0 - m), min(W, x0 + 32 + m)
        want = SV.sv_chain(xb[:, ya:yb, xa:xb_], P[:, ya:yb, xa:xb_].astype(np.float64),
                           basis.astype(np.float64), [8, 8], taps)[:, y0 - ya:y0 - ya + 32, x0 - xa:x0 - xa + 32]
        e = rel_err(got[:, y0:y0 + 32, x0:x0 + 32], want)
        print(f"sv 2d 4k bf16 crop ({y0},{x0}) halo={b.halo}: {e:.2e}")
        assert e <= TOL_BF16


@pytest.mark.parametrize("C,dims,r0,dr,want_halo", [
    (3, 1, 30.0, 3.0, [41, 41]),
    (4, 2, 30.0, 3.0, [52, 52]),
    (1, 1, 30.0, 3.0, [42, 39]),
    (3, 2, 38.0, 1.5, [43, 49]),
])
def test_sv_large_halo_global_path(dev, C, dims, r0, dr, want_halo):
    """Large halos: C = 3 at halo 41 (plane groups on the staged C <= 2
    kernel), C = 4 at halo 52 and C = 3 at 43 and 49, beyond every staged
    tile (the one-pixel-per-thread kernel), C = 1 at halos 42 and 39
    (staged)."""
    taps = [5, 6]
    G = 6 if dims == 1 else 9
    basis = _basis(G, taps, seed=500 + C, r0=r0, dr=dr)
    H, W = 96, 150
    img = noise_image(H, W, C, seed=C, n_rects=8)
    P = param_map(H, W, seed=7, period=64.0, dims=dims)
    grid = [G] if dims == 1 else [3, 3]
    say("sv large halo", C, dims, want_halo)
    out, b = _run(basis, taps, grid, img, P)
    assert list(b.halo) == want_halo
    want = SV.sv_chain(img.astype(np.float64), P.astype(np.float64), basis.astype(np.float64), grid, taps)
    e = rel_err(to_np(out), want)
    print(f"sv large halo C={C} dims={dims} halo={b.halo}: {e:.2e}")
    assert e <= TOL_F32


@pytest.mark.parametrize("C,dims,io,seed,r0,dr,want_halo", [
    (3, 1, torch.float32, 700, 24.0, 0.5, [25, 25, 27]),
    (4, 1, torch.float32, 720, 26.5, 0.5, [27, 30, 29]),
    (3, 2, torch.float32, 720, 26.5, 0.3, [28, 29, 30]),
    (3, 2, torch.bfloat16, 700, 26.0, 0.3, [28, 26, 28]),
    (3, 2, torch.float32, 800, 28.0, 0.3, [31, 29, 31]),
    (3, 2, torch.bfloat16, 820, 39.0, 0.3, [39, 40, 41]),
    (4, 2, torch.float32, 800, 39.0, 0.3, [41, 40, 42]),
    (2, 1, torch.float32, 820, 32.0, 0.5, [32, 34, 35]),
    (2, 2, torch.bfloat16, 800, 39.0, 0.3, [41, 40, 42]),
    (1, 2, torch.float32, 820, 39.0, 0.3, [39, 40, 41]),
])
def test_sv_staged_large_halo(dev, C, dims, io, seed, r0, dr, want_halo):
    """Halos 25..42 on staged tiles: C >= 3 up to halo 30 on the 8-wave kernel
    with 64 x 16 tiles and 124-pixel rows; beyond that the image's planes in
    groups of two (and one) on the 16-wave C <= 2 kernel, whose 64 x 32 tiles
    of 8-byte pixels fit up to halo 42; C <= 2 images on that kernel directly.
    Several tiles with ragged right and bottom tails, the CLAMP border on
    every side, against the oracle on the whole image."""
    taps = [6, 6, 5]
    G = 6 if dims == 1 else 9
    grid = [G] if dims == 1 else [3, 3]
    basis = _basis(G, taps, seed=seed, r0=r0, dr=dr)
    H, W = 70, 150
    img = noise_image(H, W, C, seed=seed, n_rects=10)
    P = param_map(H, W, seed=seed + 1, period=48.0, dims=dims)
    say("sv staged large halo", C, dims, io, want_halo)
    out, b = _run(basis, taps, grid, img, P, io=io)
    assert list(b.halo) == want_halo
    x = img if io == torch.float32 else bf16_round(img)
    want = SV.sv_chain(x.astype(np.float64), P.astype(np.float64), basis.astype(np.float64), grid, taps)
    e = rel_err(to_np(out), want)
    print(f"sv staged large halo C={C} dims={dims} {io} halo={b.halo}: {e:.2e}")
    assert e <= (TOL_F32 if io == torch.float32 else TOL_BF16)


def test_sv_halo_just_beyond_padded_tile(dev):
    """C = 3 with halos 31..33, just beyond the staged C >= 3 kernels (plane
    groups on the C <= 2 kernel)."""
    taps = [6, 6]
    basis = _basis(6, taps, seed=610, r0=29.6, dr=0.38)
    H, W = 80, 170
    img = noise_image(H, W, 3, seed=3, n_rects=8)
    P = param_map(H, W, seed=8, period=64.0)
    say("sv halo 31-33")
    out, b = _run(basis, taps, [6], img, P)
    assert 31 <= max(b.halo) <= 33
    want = SV.sv_chain(img.astype(np.float64), P.astype(np.float64), basis.astype(np.float64), [6], taps)
    assert rel_err(to_np(out), want) <= TOL_F32


@pytest.mark.parametrize("kind", ["rotational", "radial"])
def test_basis_rotate_and_angle_effect(dev, kind):
    """Angle axis built on the device (offsets rotated per angle, FP32)
    against the FP64 oracle's rotation, then a rotational-blur or radial
    motion-blur filter with that 2-D basis (blur length x direction) against
    the oracle."""
    from oracle import interp as IP
    from synth import direction_map
    taps = [6, 6, 6]
    base = np.stack([random_theta(taps, 1.0 + 2.0 * k, seed=700 + k) for k in range(4)]).astype(np.float32)
    angles = [np.pi * j / 8 for j in range(9)]
    say("basis rotate")
    got = disk.disk_basis_rotate(to_dev(base), angles)
    want = IP.rotate_basis(base.astype(np.float64), angles)
    assert np.abs(to_np(got) - want).max() <= 2e-6 * np.abs(want).max()
    H, W = 70, 120
    img = noise_image(H, W, 3, seed=9, n_rects=10)
    P = direction_map(H, W, kind)
    out, b = _run(to_np(got).astype(np.float32), taps, [4, 9], img, P)
    ref = SV.sv_chain(img.astype(np.float64), P.astype(np.float64), want, [4, 9], taps)
    assert rel_err(to_np(out), ref) <= TOL_F32


@pytest.mark.parametrize("C,H,W,grid,taps,io,per_frame,r0,dr", [
    (3, 150, 333, [16], [8, 8, 8, 8], torch.float32, False, 1.0, 0.8),   # pipelined kernel, frames in one launch
    (3, 97, 130, [16], [8, 8, 8, 8], torch.bfloat16, True, 1.0, 0.8),
    (4, 70, 100, [3, 3], [6, 5], torch.float32, True, 1.0, 0.8),          # 2-D basis, prepared table
    (1, 64, 80, [5], [5, 4, 6], torch.float32, False, 1.0, 0.8),          # pipelined C = 1 kernel
    (3, 70, 150, [6], [6, 6], torch.float32, True, 24.0, 0.5),            # halos 26: the wide staged kernel
    (3, 70, 150, [6], [6, 6], torch.bfloat16, False, 33.0, 0.5),          # halos 34: plane groups, per frame
    (4, 70, 150, [3, 3], [6, 5], torch.float32, True, 33.0, 0.3),         # halos 35, 36: plane groups, 2-D
])
def test_sv_frames_equal_single_frame_calls(dev, C, H, W, grid, taps, io, per_frame, r0, dr):
    """F frames in one call (one launch per pass over all frames' tiles, or a
    launch per frame and plane group for halos beyond the staged C >= 3
    kernels) equal F single-frame calls bit for bit, with one shared map or a
    map per frame."""
    F = 3
    G = int(np.prod(grid))
    b = disk.make_basis(to_dev(_basis(G, taps, seed=810 + C, r0=r0, dr=dr)), taps, grid)
    x = torch.stack([to_dev(noise_image(H, W, C, seed=H + f, n_rects=10)) for f in range(F)]).to(io)
    if per_frame:
        p = torch.stack([to_dev(param_map(H, W, seed=W + f, period=64.0, dims=len(grid))) for f in range(F)])
    else:
        p = to_dev(param_map(H, W, seed=W, period=64.0, dims=len(grid)))
    say("sv frames", C, H, W, grid, io, per_frame)
    got = disk.disk_sv_filter_frames(b, x, p)
    for f in range(F):
        # a frame's own copy: the C ABI wants 16-byte aligned buffers
        want = disk.disk_sv_filter(b, x[f].clone(), (p[f] if per_frame else p).clone())
        assert torch.equal(got[f], want), f


def test_sv_frames_bench_launch_and_graph_replay(dev):
    """The benchmark's frame batch: 32 frames of 1920 x 1080 x 3 FP32 with the
    16-entry basis of 4 x 8 taps in one call, captured into a HIP graph and
    replayed (inputs changed between replays): every replay equals the eager
    call bit for bit, the frames of one image are equal at both ends of the
    batch, and two frames equal the oracle on 96 x 96 crops with a margin of
    the summed halos."""
    taps = [8, 8, 8, 8]
    basis = _basis(16, taps, seed=300, r0=1.0, dr=0.45)
    b = disk.make_basis(to_dev(basis), taps, [16])
    H, W, F = 1080, 1920, 32
    imgs = [noise_image(H, W, 3, seed=20 + f, n_rects=50) for f in (0, 1)]
    P = param_map(H, W, seed=3)
    x = torch.stack([to_dev(imgs[f % 2]) for f in range(F)])
    p = to_dev(P)
    out = torch.empty_like(x)
    ws = disk.sv_frames_workspace(b, F, 3, H, W)
    say("sv frames 1080p x 32 eager")
    want = disk.disk_sv_filter_frames(b, x, p, ws=ws).clone()
    # frames alternate between two images: the last frames equal the first two
    assert torch.equal(want[F - 2], want[0]) and torch.equal(want[F - 1], want[1])
    say("sv frames 1080p x 32 graph capture")
    cap = disk.Captured(lambda: disk.disk_sv_filter_frames(b, x, p, out=out, ws=ws), warmup=False)
    for r in range(3):
        x[0].mul_(1.0)                       # eager work between replays
        torch.cuda.synchronize()
        say("sv frames graph replay", r)
        cap.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, want), r
    got = to_np(want)
    m = int(sum(b.halo))
    rng = np.random.default_rng(6)
    for f in (0, 1):
        y0, x0 = int(rng.integers(m, H - 96 - m)), int(rng.integers(m, W - 96 - m))
        win = (slice(y0 - m, y0 + 96 + m), slice(x0 - m, x0 + 96 + m))
        ref = SV.sv_chain(imgs[f][:, win[0], win[1]].astype(np.float64), P[:, win[0], win[1]].astype(np.float64),
                          basis.astype(np.float64), [16], taps)[:, m:m + 96, m:m + 96]
        e = rel_err(got[f][:, y0:y0 + 96, x0:x0 + 96], ref)
        print(f"frame {f} crop ({y0},{x0}): {e:.2e}")
        assert e <= TOL_F32


@pytest.mark.parametrize("seed,r0,io,want_halo", [(720, 26.5, torch.float32, [28, 29, 30]),
                                                 (820, 39.0, torch.bfloat16, [39, 40, 41])])
def test_sv_large_halo_frames_graph_replay(dev, seed, r0, io, want_halo):
    """Large-halo passes (the wide staged C = 3 kernel; plane groups, a launch
    per frame and group) captured in a HIP graph with 2 frames of a 2-D basis:
    three replays with eager work between them equal the eager call bit for
    bit."""
    taps = [6, 6, 5]
    basis = _basis(9, taps, seed=seed, r0=r0, dr=0.3)
    b = disk.make_basis(to_dev(basis), taps, [3, 3])
    assert list(b.halo) == want_halo
    H, W, F = 70, 150, 2
    x = torch.stack([to_dev(noise_image(H, W, 3, seed=seed + f, n_rects=10)) for f in range(F)]).to(io)
    p = to_dev(param_map(H, W, seed=seed + 5, period=48.0, dims=2))
    out = torch.empty_like(x)
    ws = disk.sv_frames_workspace(b, F, 3, H, W, disk.BF16 if io == torch.bfloat16 else disk.F32)
    say("sv large halo frames eager", want_halo, io)
    want = disk.disk_sv_filter_frames(b, x, p, ws=ws).clone()
    say("sv large halo frames graph capture")
    cap = disk.Captured(lambda: disk.disk_sv_filter_frames(b, x, p, out=out, ws=ws), warmup=False)
    for r in range(3):
        x[0].mul_(1.0)                       # eager work between replays
        torch.cuda.synchronize()
        say("sv large halo graph replay", r)
        cap.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, want), r


def test_tilt_shift_from_pseudo_depth(dev):
    """Tilt-shift (the depth-driven effect of the paper's spatially varying
    examples): blur from the distance of a pseudo-depth map to the focal
    depth, with a disk-like 1-D basis of 16 entries (4 x 8 taps).  A 96 x 160
    image against the oracle in full, and the 1920 x 1080 frame on a
    top-border crop, a bottom-corner crop and an interior crop, each with a
    margin of the summed halos (clipped at the image's edges, which the
    oracle treats as the same CLAMP border)."""
    from synth import tilt_shift_map
    taps = [8, 8, 8, 8]
    basis = _basis(16, taps, seed=320, r0=0.8, dr=0.5)
    H, W = 96, 160
    img = noise_image(H, W, 3, seed=31, n_rects=12)
    P = tilt_shift_map(H, W, seed=5)
    say("tilt-shift small")
    out, b = _run(basis, taps, [16], img, P)
    want = SV.sv_chain(img.astype(np.float64), P.astype(np.float64), basis.astype(np.float64), [16], taps)
    assert rel_err(to_np(out), want) <= TOL_F32
    H, W = 1080, 1920
    img = noise_image(H, W, 3, seed=32, n_rects=60)
    P = tilt_shift_map(H, W)
    say("tilt-shift 1080p")
    out, b = _run(basis, taps, [16], img, P)
    got = to_np(out)
    m = int(sum(b.halo))
    for y0, x0 in ((0, 700), (H - 64, W - 64), (500, 900)):
        ya, yb, xa, xb = max(0, y0 - m), min(H, y0 + 64 + m), max(0, x0 - m), min(W, x0 + 64 + m)
        ref = SV.sv_chain(img[:, ya:yb, xa:xb].astype(np.float64), P[:, ya:yb, xa:xb].astype(np.float64),
                          basis.astype(np.float64), [16], taps)[:, y0 - ya:y0 - ya + 64, x0 - xa:x0 - xa + 64]
        e = rel_err(got[:, y0:y0 + 64, x0:x0 + 64], ref)
        print(f"tilt-shift 1080p crop ({y0},{x0}): {e:.2e}")
        assert e <= TOL_F32
