"""The allocation-free entry point disk_sv_filter_noalloc (scratch in the
library's fixed device array) against disk_sv_filter with a caller workspace,
through the C ABI: two calls in a row, the second on a smaller input (and on
the prepared-table path of a 2-D basis, whose table also lives in the
array), each equal to the workspace entry point bit for bit; a frame whose
scratch exceeds the array is refused before anything is launched."""
import numpy as np
import pytest
import torch

import paper_2512_04556_amd as disk
from synth import random_theta, noise_image, param_map
from tests.gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


def _basis(G, taps, seed, r0, dr):
    return np.stack([random_theta(taps, r0 + dr * k, seed=seed + k) for k in range(G)]).astype(np.float32)


def test_noalloc_matches_workspace_entry_point(dev):
    cases = [
        # the benchmark frame: 1920 x 1080 x 3 FP32, 16-entry 1-D basis, 4 x 8 taps
        (3, 1080, 1920, [16], [8, 8, 8, 8], torch.float32, 1.0, 0.7),
        # smaller, 2-D 3 x 3 basis (prepared table in the array), BF16 I/O
        (3, 97, 130, [3, 3], [6, 5, 7], torch.bfloat16, 1.5, 0.8),
    ]
    for C, H, W, grid, taps, io, r0, dr in cases:
        G = int(np.prod(grid))
        b = disk.make_basis(to_dev(_basis(G, taps, 900 + G, r0, dr)), taps, grid)
        x = to_dev(noise_image(H, W, C, seed=H)).to(io)
        p = to_dev(param_map(H, W, seed=W, period=64.0, dims=len(grid)))
        want = disk.disk_sv_filter(b, x, p)
        got = torch.full_like(x, float("nan"))
        say("sv noalloc", C, H, W, grid, io)
        disk.disk_sv_filter_noalloc(b, x, p, got)
        torch.cuda.synchronize()
        assert torch.equal(got, want), (H, W, grid)
        print(f"noalloc {C}x{H}x{W} grid {grid} {io}: bitwise equal to disk_sv_filter")


def test_noalloc_refuses_frames_beyond_the_array(dev):
    taps = [4, 4]
    b = disk.make_basis(to_dev(_basis(2, taps, 950, 1.0, 1.0)), taps, [2])
    C, H, W = 3, 2160, 3840
    need = disk.lib().disk_sv_filter_workspace_size(disk.ctypes.byref(b.desc), C, H, W, disk.F32)
    assert need > disk.lib().disk_sv_noalloc_max_bytes()
    x = torch.zeros((C, H, W), device="cuda")
    p = torch.zeros((1, H, W), device="cuda")
    out = torch.zeros_like(x)
    with pytest.raises(disk.DiskError, match="scratch"):
        disk.disk_sv_filter_noalloc(b, x, p, out)
    assert int(torch.count_nonzero(out)) == 0
