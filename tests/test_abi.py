"""CPU checks of the C ABI: the library loads, exports every entry point that
include/disk.h declares, and rejects bad arguments before enqueuing any work
(no GPU needed for any call here)."""
import ctypes
import os
import re

import pytest

import paper_2512_04556_amd as disk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "disk.h")


def _declared():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(disk_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    L = disk.lib()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n


def test_status_strings_and_version():
    L = disk.lib()
    assert L.disk_status_string(0) == b"DISK_OK"
    assert L.disk_status_string(-3) == b"DISK_WORKSPACE_TOO_SMALL"
    assert b"gfx950" in L.disk_version()


def _cx(taps):
    return disk._complex(taps)


def test_forward_validation_fails_before_launch():
    L = disk.lib()
    P = ctypes.c_void_p
    fake = P(0x1000)           # aligned, never dereferenced: validation fails first
    cx = _cx([8, 8])
    # L out of range
    bad = disk.DiskComplex()
    bad.L = 9
    assert L.disk_forward(ctypes.byref(bad), fake, fake, fake, 1, 8, 8, 0, 1, None, fake, 1 << 20, None) == -2
    # taps out of range
    bad2 = _cx([8])
    bad2.taps[0] = 33
    assert L.disk_forward(ctypes.byref(bad2), fake, fake, fake, 1, 8, 8, 0, 1, None, fake, 1 << 20, None) == -2
    # null theta
    assert L.disk_forward(ctypes.byref(cx), None, fake, fake, 1, 8, 8, 0, 1, None, fake, 1 << 20, None) == -1
    assert b"theta" in L.disk_last_error()
    # misaligned pointer
    assert L.disk_forward(ctypes.byref(cx), P(0x1004), fake, fake, 1, 8, 8, 0, 1, None, fake, 1 << 20, None) == -1
    # C out of range
    assert L.disk_forward(ctypes.byref(cx), fake, fake, fake, 5, 8, 8, 0, 1, None, fake, 1 << 20, None) == -2
    # impulse mode: even side, C != 1, CLAMP
    assert L.disk_forward(ctypes.byref(cx), fake, None, fake, 1, 8, 9, 0, 0, None, fake, 1 << 20, None) == -2
    assert L.disk_forward(ctypes.byref(cx), fake, None, fake, 2, 9, 9, 0, 0, None, fake, 1 << 20, None) == -2
    assert L.disk_forward(ctypes.byref(cx), fake, None, fake, 1, 9, 9, 0, 1, None, fake, 1 << 20, None) == -1
    # workspace too small
    need = L.disk_forward_workspace_size(ctypes.byref(cx), 3, 64, 64, 0, 0, 0)
    assert need > 3 * 64 * 64 * 4
    assert L.disk_forward(ctypes.byref(cx), fake, fake, fake, 3, 64, 64, 0, 1, None, fake, need - 4096, None) == -3


def test_backward_and_sv_validation():
    L = disk.lib()
    P = ctypes.c_void_p
    fake = P(0x1000)
    cx = _cx([4, 4])
    # saved required for L > 1
    assert L.disk_backward(ctypes.byref(cx), fake, fake, None, fake, fake, fake, 1, 8, 8, 1, fake, 1 << 20, None) == -1
    b = disk.DiskBasis()
    b.dims = 3
    assert L.disk_sv_filter(ctypes.byref(b), fake, fake, fake, fake, 3, 8, 8, 0, fake, 1 << 20, None) == -2
    b.dims = 1
    b.grid[0] = 4
    b.cx = _cx([4, 4])
    b.halo[0] = 0
    b.halo[1] = 3
    assert L.disk_sv_filter(ctypes.byref(b), fake, fake, fake, P(0x2000), 3, 8, 8, 0, fake, 1 << 20, None) == -5
    b.halo[0] = 3
    other = P(0x2000)
    assert L.disk_sv_filter(ctypes.byref(b), fake, fake, fake, other, 3, 8, 8, 0, None, 0, None) == -3
    # image aliasing out
    assert L.disk_sv_filter(ctypes.byref(b), fake, fake, fake, fake, 3, 8, 8, 0, fake, 1 << 20, None) == -1
    # frames: count out of range, aliasing, workspace sized for all frames
    for F in (0, 65):
        assert L.disk_sv_filter_frames(ctypes.byref(b), fake, fake, fake, 0, other, F, 3, 8, 8, 0, fake, 1 << 20,
                                       None) == -2
        assert L.disk_sv_filter_frames_workspace_size(ctypes.byref(b), F, 3, 8, 8, 0) == 0
    assert L.disk_sv_filter_frames(ctypes.byref(b), fake, fake, fake, 1, fake, 2, 3, 8, 8, 0, fake, 1 << 20,
                                   None) == -1
    one = L.disk_sv_filter_frames_workspace_size(ctypes.byref(b), 1, 3, 64, 64, 0)
    eight = L.disk_sv_filter_frames_workspace_size(ctypes.byref(b), 8, 3, 64, 64, 0)
    assert one == L.disk_sv_filter_workspace_size(ctypes.byref(b), 3, 64, 64, 0)
    assert eight > 7 * (one - L.disk_sv_table_bytes(ctypes.byref(b)) - 256)
    assert L.disk_sv_filter_frames(ctypes.byref(b), fake, fake, fake, 0, other, 8, 3, 64, 64, 0, fake, one,
                                   None) == -3
    # the allocation-free filter refuses frames whose scratch exceeds its fixed array
    assert L.disk_sv_filter_noalloc(ctypes.byref(b), fake, fake, fake, other, 3, 2160, 3840, 0, None) == -3
    assert b"scratch" in L.disk_last_error()


def test_basis_halo_from_host_copy():
    import torch
    taps = [3, 2]
    th = torch.zeros((2, 5, 3))
    th[0, 0, 0] = 4.0          # layer 0: max |o| = 4  -> halo 5
    th[1, 1, 1] = -2.5         # layer 0: 2.5
    th[1, 3, 0] = 7.25         # layer 1: 7.25 -> halo 9
    b = disk.Basis.__new__(disk.Basis)
    d = disk.DiskBasis()
    d.dims = 1
    d.grid[0] = 2
    d.cx = _cx(taps)
    host = th.contiguous()
    assert disk.lib().disk_basis_set_halo(ctypes.byref(d), ctypes.c_void_p(host.data_ptr())) == 0
    assert [d.halo[0], d.halo[1]] == [5, 9]
    th[0, 2, 2] = float("nan")
    assert disk.lib().disk_basis_set_halo(ctypes.byref(d), ctypes.c_void_p(host.data_ptr())) == -1


def test_optimiser_and_basis_fit_validation():
    L = disk.lib()
    P = ctypes.c_void_p
    fake = P(0x1000)
    meta = disk.DiskBatchMeta(4, 31, 24)
    prm = disk.OptParams(max_steps=10).c
    sc = (ctypes.c_float * 4)(1.0, 2.0, 1.5, 1.2)
    ws = 1 << 30
    args = (ctypes.byref(meta), fake, fake, fake, fake, fake, fake, fake)
    # even max_side, B < 1
    bad = disk.DiskBatchMeta(4, 30, 24)
    assert L.disk_optimize_batch(ctypes.byref(bad), *args[1:], None, ctypes.byref(prm), None, None, fake, ws,
                                 None) == -2
    assert L.disk_fit_basis(ctypes.byref(disk.DiskBatchMeta(0, 31, 24)), *args[1:], sc, ctypes.byref(prm),
                            fake, ws, None) == -2
    # scale missing or not positive
    assert L.disk_fit_basis(*args, None, ctypes.byref(prm), fake, ws, None) == -1
    sc_bad = (ctypes.c_float * 4)(1.0, 2.0, 0.0, 1.2)
    assert L.disk_fit_basis(*args, sc_bad, ctypes.byref(prm), fake, ws, None) == -1
    assert b"scale[2]" in L.disk_last_error()
    # Adam hyper-parameters
    bad_p = disk.OptParams(max_steps=10, beta1=1.0).c
    assert L.disk_fit_basis(*args, sc, ctypes.byref(bad_p), fake, ws, None) == -1
    assert L.disk_optimize_batch(*args, None, ctypes.byref(bad_p), None, None, fake, ws, None) == -1
    bad_u = disk.OptParams(max_steps=10, offset_units=2).c
    assert L.disk_optimize_batch(*args, None, ctypes.byref(bad_u), None, None, fake, ws, None) == -1
    assert b"offset_units" in L.disk_last_error()
    # misaligned finish_ticks
    assert L.disk_optimize_batch(*args, P(0x1008), ctypes.byref(prm), None, None, fake, ws, None) == -1
    # launch shape out of range; Adam moments given without the other
    for th, w in ((256, 0), (256, 5), (1024, 2), (512, 1)):
        tune = disk.DiskOptTune(th, w)
        assert L.disk_optimize_batch(*args, None, ctypes.byref(prm), None, ctypes.byref(tune), fake, ws, None) == -1
        assert L.disk_optimize_workspace_size(ctypes.byref(meta), ctypes.byref(tune)) == 0
    st = disk.DiskOptState(fake, None, None, None, 0)
    assert L.disk_optimize_batch(*args, None, ctypes.byref(prm), ctypes.byref(st), None, fake, ws, None) == -1
    st = disk.DiskOptState(fake, fake, None, None, -1)
    assert L.disk_optimize_batch(*args, None, ctypes.byref(prm), ctypes.byref(st), None, fake, ws, None) == -1
    # more resident work-groups need more workspace
    t1, t4 = disk.DiskOptTune(256, 1), disk.DiskOptTune(256, 4)
    assert (L.disk_optimize_workspace_size(ctypes.byref(meta), ctypes.byref(t1)) <=
            L.disk_optimize_workspace_size(ctypes.byref(meta), ctypes.byref(t4)))
    # workspace too small
    need = L.disk_fit_basis_workspace_size(ctypes.byref(meta))
    assert need > 0
    assert L.disk_fit_basis(*args, sc, ctypes.byref(prm), fake, need - 512, None) == -3
