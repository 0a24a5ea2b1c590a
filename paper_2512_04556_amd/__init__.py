"""Python binding of libdisk (ctypes): argument marshalling only.

Every function forwards to the C entry point of the same name in libdisk.so
(declared in include/disk.h); torch supplies device memory (outputs and the
workspace each call needs) and the current stream.  There is no fallback: if
libdisk.so is missing, or a tensor is not on the GPU, the call raises.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_float, c_int32, c_int64, c_size_t, c_uint64, c_void_p

import torch

__all__ = [
    "lib", "DiskError", "ZERO", "CLAMP", "F32", "BF16", "LOSS_NMSE", "LOSS_CHARBONNIER",
    "disk_forward", "disk_backward", "disk_sv_filter", "disk_sv_filter_frames", "sv_frames_workspace", "disk_sv_filter_noalloc",
    "disk_sv_prepare", "disk_sv_apply", "Basis", "make_basis",
    "disk_optimize_batch", "Captured", "OptState", "opt_tune", "optimize_workspace_size", "OFFSETS_PIXELS",
    "OFFSETS_HALF_WIDTH", "disk_init_radial", "disk_init_random", "disk_fit_basis", "pack_targets", "fit_basis", "disk_init_shape", "OptParams", "Batch", "make_batch",
    "disk_init_predict", "disk_net_train_step", "disk_net_prepare_inputs", "disk_net_scatter_theta",
    "disk_net_param_count", "net_workspace", "clock_rate_khz",
    "disk_dense_sv", "DENSE_DISK", "DENSE_ELLIPSE", "disk_basis_rotate",
]

ZERO, CLAMP = 0, 1
F32, BF16 = 0, 1
LOSS_NMSE, LOSS_CHARBONNIER = 0, 1
MAX_LAYERS = 8

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


class DiskError(RuntimeError):
    pass


class DiskComplex(ctypes.Structure):
    _fields_ = [("L", c_int32), ("taps", c_int32 * MAX_LAYERS)]


class DiskBasis(ctypes.Structure):
    _fields_ = [("dims", c_int32), ("grid", c_int32 * 2), ("cx", DiskComplex), ("halo", c_int32 * MAX_LAYERS)]


class DiskOptParams(ctypes.Structure):
    _fields_ = [("max_steps", c_int32), ("lr0", c_float), ("lr1", c_float), ("beta1", c_float),
                ("beta2", c_float), ("eps", c_float), ("psnr_stop_db", c_float), ("loss", c_int32),
                ("charb_eps", c_float), ("offset_units", c_int32)]


class DiskOptState(ctypes.Structure):
    _fields_ = [("adam_m", c_void_p), ("adam_v", c_void_p), ("start_step", c_void_p), ("loss", c_void_p),
                ("max_updates", c_int32)]


class DiskOptTune(ctypes.Structure):
    _fields_ = [("threads", c_int32), ("wgs_per_cu", c_int32)]


class DiskDenseParams(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("r0", c_float), ("r1", c_float), ("a0", c_float), ("a1", c_float),
                ("half", c_int32)]


class DiskBatchMeta(ctypes.Structure):
    _fields_ = [("B", c_int32), ("max_side", c_int32), ("max_T", c_int32)]


def lib():
    """Load libdisk.so from the package directory (raises if it was not built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = os.path.join(_HERE, "libdisk.so")
    if not os.path.exists(path):
        raise DiskError(f"{path} is missing: build it with `python -m paper_2512_04556_amd.build`")
    L = ctypes.CDLL(path)
    P = c_void_p
    sig = {
        "disk_status_string": (ctypes.c_char_p, [c_int32]),
        "disk_last_error": (ctypes.c_char_p, []),
        "disk_version": (ctypes.c_char_p, []),
        "disk_forward_workspace_size": (c_size_t, [POINTER(DiskComplex), c_int32, c_int32, c_int32, c_int32, c_int32, c_int32]),
        "disk_forward": (c_int32, [POINTER(DiskComplex), P, P, P, c_int32, c_int32, c_int32, c_int32, c_int32, P, P, c_size_t, P]),
        "disk_backward_workspace_size": (c_size_t, [POINTER(DiskComplex), c_int32, c_int32, c_int32]),
        "disk_backward": (c_int32, [POINTER(DiskComplex), P, P, P, P, P, P, c_int32, c_int32, c_int32, c_int32, P, c_size_t, P]),
        "disk_optimize_workspace_size": (c_size_t, [POINTER(DiskBatchMeta), POINTER(DiskOptTune)]),
        "disk_optimize_default_tune": (c_int32, [POINTER(DiskBatchMeta), POINTER(DiskOptTune)]),
        "disk_optimize_batch": (c_int32, [POINTER(DiskBatchMeta), P, P, P, P, P, P, P, P, POINTER(DiskOptParams),
                                          POINTER(DiskOptState), POINTER(DiskOptTune), P, c_size_t, P]),
        "disk_clock_rate_khz": (c_int64, []),
        "disk_basis_rotate": (c_int32, [P, c_int32, c_int32, POINTER(c_double), c_int32, P, P]),
        "disk_dense_sv": (c_int32, [POINTER(DiskDenseParams), P, P, P, c_int32, c_int32, c_int32, c_int32, P]),
        "disk_init_radial": (c_int32, [POINTER(DiskBatchMeta), P, P, P, P, P]),
        "disk_fit_basis_workspace_size": (c_size_t, [POINTER(DiskBatchMeta)]),
        "disk_fit_basis": (c_int32, [POINTER(DiskBatchMeta), P, P, P, P, P, P, P, POINTER(c_float),
                                     POINTER(DiskOptParams), P, c_size_t, P]),
        "disk_init_shape": (c_int32, [P, c_int32, c_int32, P, c_uint64, c_int32, P, POINTER(c_double)]),
        "disk_init_random": (c_int32, [P, c_int32, c_int32, P, c_uint64, c_int32, P, POINTER(c_double)]),
        "disk_basis_set_halo": (c_int32, [POINTER(DiskBasis), P]),
        "disk_sv_filter_workspace_size": (c_size_t, [POINTER(DiskBasis), c_int32, c_int32, c_int32, c_int32]),
        "disk_sv_filter": (c_int32, [POINTER(DiskBasis), P, P, P, P, c_int32, c_int32, c_int32, c_int32, P, c_size_t, P]),
        "disk_sv_filter_frames_workspace_size": (c_size_t, [POINTER(DiskBasis), c_int32, c_int32, c_int32, c_int32,
                                                            c_int32]),
        "disk_sv_filter_frames": (c_int32, [POINTER(DiskBasis), P, P, P, c_int32, P, c_int32, c_int32, c_int32,
                                            c_int32, c_int32, P, c_size_t, P]),
        "disk_sv_noalloc_max_bytes": (c_size_t, []),
        "disk_sv_filter_noalloc": (c_int32, [POINTER(DiskBasis), P, P, P, P, c_int32, c_int32, c_int32, c_int32, P]),
        "disk_sv_table_bytes": (c_size_t, [POINTER(DiskBasis)]),
        "disk_sv_prepare": (c_int32, [POINTER(DiskBasis), P, P, c_size_t, P]),
        "disk_sv_apply_workspace_size": (c_size_t, [POINTER(DiskBasis), c_int32, c_int32, c_int32, c_int32]),
        "disk_sv_apply": (c_int32, [POINTER(DiskBasis), P, P, P, P, c_int32, c_int32, c_int32, c_int32, P, c_size_t, P]),
        "disk_net_param_count": (c_int64, []),
        "disk_net_workspace_size": (c_size_t, [c_int32]),
        "disk_net_predict_workspace_size": (c_size_t, [c_int32]),
        "disk_init_predict": (c_int32, [P, P, P, P, c_int32, P, c_size_t, P]),
        "disk_net_train_step": (c_int32, [P, P, P, c_int32, c_float, P, P, P, c_int32, P, P, P, c_size_t, P]),
        "disk_net_prepare_inputs": (c_int32, [POINTER(DiskBatchMeta), P, P, P, P, P]),
        "disk_net_scatter_theta": (c_int32, [POINTER(DiskBatchMeta), P, P, P, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = L
    return L


def _check(status: int):
    if status != 0:
        L = lib()
        raise DiskError(f"{L.disk_status_string(status).decode()}: {L.disk_last_error().decode()}")


def _ptr(t):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch.Tensor")
    if not t.is_contiguous():
        raise DiskError("tensor must be contiguous")
    return c_void_p(t.data_ptr())


def _dev(t, name):
    if t is not None and not t.is_cuda:
        raise DiskError(f"{name} must be a GPU tensor")


def _f32(t, name):
    """The C entry points read these as float*: refuse any other dtype."""
    if t is not None and t.dtype != torch.float32:
        raise DiskError(f"{name} must be float32 (got {t.dtype})")


def _stream():
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def _complex(taps):
    taps = [int(t) for t in taps]
    cx = DiskComplex()
    cx.L = len(taps)
    if not 1 <= cx.L <= MAX_LAYERS:
        raise DiskError(f"L={cx.L} out of range")
    for i, t in enumerate(taps):
        cx.taps[i] = t
    return cx


def _workspace(nbytes, device):
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def _io_dtype(t):
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.bfloat16:
        return BF16
    raise DiskError(f"unsupported image dtype {t.dtype}")


# ---------------------------------------------------------------------------
def disk_forward(theta, taps, inp=None, *, H=None, W=None, boundary=CLAMP, save=False, out=None):
    """Chain forward.  ``inp`` [C][H][W] (f32/bf16) or None for the impulse
    response on an H x W canvas.  Returns (out, saved) with saved the
    intermediates [(L-1)][C][H][W] when ``save``."""
    _dev(theta, "theta")
    _f32(theta, "theta")
    dev = theta.device
    cx = _complex(taps)
    if inp is None:
        C, io, impulse = 1, F32, 1
        H = int(H)
        W = int(W if W is not None else H)
        boundary = ZERO
    else:
        _dev(inp, "inp")
        C, H, W = inp.shape
        io, impulse = _io_dtype(inp), 0
    if out is None:
        out = torch.empty((C, H, W), dtype=torch.float32 if io == F32 else torch.bfloat16, device=dev)
    saved = torch.empty((max(cx.L - 1, 1), C, H, W), dtype=torch.float32, device=dev) if save else None
    L = lib()
    nws = L.disk_forward_workspace_size(ctypes.byref(cx), C, H, W, io, impulse, int(save))
    ws = _workspace(nws, dev)
    _check(L.disk_forward(ctypes.byref(cx), _ptr(theta), _ptr(inp), _ptr(out), C, H, W, io, boundary,
                          _ptr(saved) if save else None, _ptr(ws), ws.numel(), _stream()))
    return out, saved


def disk_backward(theta, taps, inp, saved, grad_out, *, boundary=CLAMP, need_theta=True, need_input=True):
    """Adjoint.  Returns (grad_theta [T][3] or None, grad_in [C][H][W] or None)."""
    _dev(theta, "theta")
    _dev(grad_out, "grad_out")
    _dev(inp, "inp")
    _dev(saved, "saved")
    # the C entry point reads every one of these as float*
    _f32(theta, "theta")
    _f32(grad_out, "grad_out")
    _f32(inp, "inp")
    _f32(saved, "saved")
    dev = theta.device
    cx = _complex(taps)
    if grad_out.dim() != 3:
        raise DiskError(f"grad_out must be [C][H][W] (got shape {tuple(grad_out.shape)})")
    C, H, W = (int(v) for v in grad_out.shape)
    T = sum(int(t) for t in taps)
    if tuple(theta.shape) != (T, 3):
        raise DiskError(f"theta must be [{T}][3] (got {tuple(theta.shape)})")
    if inp is not None and tuple(inp.shape) != (C, H, W):
        raise DiskError(f"inp shape {tuple(inp.shape)} differs from grad_out shape {(C, H, W)}")
    if cx.L > 1:
        if saved is None or saved.dim() != 4 or tuple(saved.shape[1:]) != (C, H, W) or saved.shape[0] < cx.L - 1:
            raise DiskError(f"saved must be [{cx.L - 1}][{C}][{H}][{W}] "
                            f"(got {None if saved is None else tuple(saved.shape)})")
    if inp is None:
        boundary = ZERO
    gt = torch.empty_like(theta) if need_theta else None
    gi = torch.empty((C, H, W), dtype=torch.float32, device=dev) if need_input else None
    L = lib()
    ws = _workspace(L.disk_backward_workspace_size(ctypes.byref(cx), C, H, W), dev)
    _check(L.disk_backward(ctypes.byref(cx), _ptr(theta), _ptr(inp), _ptr(saved), _ptr(grad_out), _ptr(gt),
                           _ptr(gi), C, H, W, boundary, _ptr(ws), ws.numel(), _stream()))
    return gt, gi


# ---------------------------------------------------------------------------
class Basis:
    """A filter-space basis: device tensor [G][T][3] plus its C descriptor."""

    def __init__(self, theta, taps, grid):
        _f32(theta, "basis theta")
        self.theta = theta.contiguous()
        self.taps = [int(t) for t in taps]
        self.grid = [int(g) for g in grid]
        d = DiskBasis()
        d.dims = len(self.grid)
        d.grid[0] = self.grid[0]
        d.grid[1] = self.grid[1] if len(self.grid) > 1 else 1
        d.cx = _complex(self.taps)
        host = self.theta.detach().to("cpu", torch.float32).contiguous()
        _check(lib().disk_basis_set_halo(ctypes.byref(d), _ptr(host)))
        self.desc = d

    @property
    def halo(self):
        return [self.desc.halo[l] for l in range(len(self.taps))]


def make_basis(theta, taps, grid):
    return Basis(theta, taps, grid)


def disk_sv_filter(basis: Basis, image, pmap, out=None, ws=None):
    """Spatially varying filter of ``image`` [C][H][W] (f32/bf16) with the
    per-pixel parameters ``pmap`` [dims][H][W] (f32)."""
    _dev(image, "image")
    _dev(pmap, "pmap")
    _f32(pmap, "pmap")
    C, H, W = image.shape
    io = _io_dtype(image)
    if out is None:
        out = torch.empty_like(image)
    L = lib()
    nws = L.disk_sv_filter_workspace_size(ctypes.byref(basis.desc), C, H, W, io)
    if ws is None or ws.numel() < nws:
        ws = _workspace(nws, image.device)
    _check(L.disk_sv_filter(ctypes.byref(basis.desc), _ptr(basis.theta), _ptr(image), _ptr(pmap), _ptr(out),
                            C, H, W, io, _ptr(ws), ws.numel(), _stream()))
    return out


def disk_sv_filter_frames(basis: Basis, images, pmaps, out=None, ws=None):
    """The filter over F frames in one call: ``images`` [F][C][H][W]
    (f32/bf16); ``pmaps`` [dims][H][W] (shared by every frame) or
    [F][dims][H][W]."""
    _dev(images, "images")
    _dev(pmaps, "pmaps")
    _f32(pmaps, "pmaps")
    if images.dim() != 4:
        raise DiskError("images must be [F][C][H][W]")
    F, C, H, W = (int(v) for v in images.shape)
    per_frame = pmaps.dim() == 4
    if (per_frame and (int(pmaps.shape[0]) != F or tuple(pmaps.shape[2:]) != (H, W))) or \
            (not per_frame and tuple(pmaps.shape[1:]) != (H, W)):
        raise DiskError(f"pmaps shape {tuple(pmaps.shape)} does not fit images {tuple(images.shape)}")
    io = _io_dtype(images)
    if out is None:
        out = torch.empty_like(images)
    L = lib()
    nws = L.disk_sv_filter_frames_workspace_size(ctypes.byref(basis.desc), F, C, H, W, io)
    if ws is None or ws.numel() < nws:
        ws = _workspace(nws, images.device)
    _check(L.disk_sv_filter_frames(ctypes.byref(basis.desc), _ptr(basis.theta), _ptr(images), _ptr(pmaps),
                                   int(per_frame), _ptr(out), F, C, H, W, io, _ptr(ws), ws.numel(), _stream()))
    return out


def sv_frames_workspace(basis: Basis, F, C, H, W, io=F32, device="cuda"):
    return _workspace(lib().disk_sv_filter_frames_workspace_size(ctypes.byref(basis.desc), F, C, H, W, io), device)


def disk_sv_filter_noalloc(basis: Basis, image, pmap, out):
    """disk_sv_filter without a workspace: the library's fixed device array
    holds the scratch (calls on one GPU must not overlap).  ``out`` is
    required, so the call allocates nothing."""
    _dev(image, "image")
    _dev(pmap, "pmap")
    _dev(out, "out")
    _f32(pmap, "pmap")
    if out.dtype != image.dtype or tuple(out.shape) != tuple(image.shape):
        raise DiskError("out must match the image's dtype and shape")
    C, H, W = image.shape
    _check(lib().disk_sv_filter_noalloc(ctypes.byref(basis.desc), _ptr(basis.theta), _ptr(image), _ptr(pmap),
                                        _ptr(out), C, H, W, _io_dtype(image), _stream()))
    return out


def sv_filter_workspace(basis: Basis, C, H, W, io=F32, device="cuda"):
    nws = lib().disk_sv_filter_workspace_size(ctypes.byref(basis.desc), C, H, W, io)
    return _workspace(nws, device)


def disk_sv_prepare(basis: Basis, table=None):
    """Coefficient table of a basis (device uint8 tensor), for disk_sv_apply."""
    L = lib()
    nb = L.disk_sv_table_bytes(ctypes.byref(basis.desc))
    if table is None or table.numel() < nb:
        table = _workspace(nb, basis.theta.device)
    _check(L.disk_sv_prepare(ctypes.byref(basis.desc), _ptr(basis.theta), _ptr(table), table.numel(), _stream()))
    return table


def disk_sv_apply(basis: Basis, table, image, pmap, out=None, ws=None):
    """The L passes of the SV filter with a prepared table."""
    _dev(image, "image")
    _dev(pmap, "pmap")
    _f32(pmap, "pmap")
    C, H, W = image.shape
    io = _io_dtype(image)
    if out is None:
        out = torch.empty_like(image)
    L = lib()
    nws = L.disk_sv_apply_workspace_size(ctypes.byref(basis.desc), C, H, W, io)
    if ws is None or ws.numel() < nws:
        ws = _workspace(nws, image.device)
    _check(L.disk_sv_apply(ctypes.byref(basis.desc), _ptr(table), _ptr(image), _ptr(pmap), _ptr(out), C, H, W, io,
                           _ptr(ws), ws.numel(), _stream()))
    return out


# ---------------------------------------------------------------------------
# batched optimisation and initialisers
# ---------------------------------------------------------------------------
OFFSETS_PIXELS, OFFSETS_HALF_WIDTH = 0, 1


class OptParams:
    def __init__(self, max_steps=1000, lr0=1e-2, lr1=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                 psnr_stop_db=float("inf"), loss=LOSS_NMSE, charb_eps=1e-3, offset_units=OFFSETS_PIXELS):
        self.c = DiskOptParams(int(max_steps), lr0, lr1, beta1, beta2, eps, psnr_stop_db, int(loss), charb_eps,
                               int(offset_units))


class OptState:
    """Adam state carried across disk_optimize_batch calls (resume), the loss
    of the returned Theta, and a cap on the updates of one call.  adam_m,
    adam_v: float32 [*][3] like theta (in/out, given together or not at all);
    start_step: int32 [B] (in); loss: float32 [B] (out)."""

    def __init__(self, adam_m=None, adam_v=None, start_step=None, loss=None, max_updates=0):
        for t, name in ((adam_m, "adam_m"), (adam_v, "adam_v"), (loss, "loss")):
            _dev(t, name)
            _f32(t, name)
        _dev(start_step, "start_step")
        if start_step is not None and start_step.dtype != torch.int32:
            raise DiskError("start_step must be int32")
        self.tensors = (adam_m, adam_v, start_step, loss)
        self.c = DiskOptState(*[None if t is None else _ptr(t) for t in self.tensors], int(max_updates))


def opt_tune(wgs_per_cu, threads=256):
    """A launch shape for disk_optimize_batch (None selects the built-in table):
    256 threads with 1..4 work-groups per CU, or 1024 threads with 1."""
    return DiskOptTune(int(threads), int(wgs_per_cu))


class Batch:
    """Packed batch of targets on the device (layout of disk_target)."""

    def __init__(self, desc, taps, targets, max_side, max_T):
        self.desc = desc          # int32 [B][5] device
        self.taps = taps          # int32 device
        self.targets = targets    # float32 device
        self.meta = DiskBatchMeta(int(desc.shape[0]), int(max_side), int(max_T))
        self.T_total = None

    @property
    def B(self):
        return self.meta.B


def make_batch(desc, taps, targets, device="cuda"):
    """desc int32 [B][5] = (side, L, taps_off, theta_off, target_off) (numpy or
    tensor), taps int32, targets float32 (packed kernels)."""
    d = torch.as_tensor(desc, dtype=torch.int32)
    tp = torch.as_tensor(taps, dtype=torch.int32)
    tg = torch.as_tensor(targets, dtype=torch.float32)
    max_side = int(d[:, 0].max())
    Ts = [int(tp[int(d[b, 2]):int(d[b, 2]) + int(d[b, 1])].sum()) for b in range(d.shape[0])]
    bt = Batch(d.to(device).contiguous(), tp.to(device).contiguous(), tg.to(device).contiguous(), max_side, max(Ts))
    bt.T_total = int(max(int(d[b, 3]) + Ts[b] for b in range(d.shape[0])))
    return bt


def disk_optimize_batch(batch: Batch, theta, params: OptParams, ticks=None, state: OptState = None, tune=None,
                        ws=None):
    """Optimise every target of ``batch`` in place on ``theta`` [*][3].
    Returns (psnr_db [B], steps [B], status [B]).  ``ticks`` (optional,
    int64 [B + 1]) receives the device clock at each target's finish and, in
    entry B, at the launch's start.  ``state``: an OptState (resume, loss);
    ``tune``: opt_tune(...) or None for the built-in table; ``ws``: a
    workspace to reuse (uint8, at least optimize_workspace_size bytes)."""
    _dev(theta, "theta")
    _f32(theta, "theta")
    dev = theta.device
    B = batch.B
    psnr = torch.empty(B, dtype=torch.float32, device=dev)
    steps = torch.empty(B, dtype=torch.int32, device=dev)
    status = torch.empty(B, dtype=torch.int32, device=dev)
    L = lib()
    tn = None if tune is None else ctypes.byref(tune)
    if ws is None:
        ws = _workspace(L.disk_optimize_workspace_size(ctypes.byref(batch.meta), tn), dev)
    st = None if state is None else ctypes.byref(state.c)
    _check(L.disk_optimize_batch(ctypes.byref(batch.meta), _ptr(batch.desc), _ptr(batch.taps), _ptr(batch.targets),
                                 _ptr(theta), _ptr(psnr), _ptr(steps), _ptr(status), _ptr(ticks),
                                 ctypes.byref(params.c), st, tn, _ptr(ws), ws.numel(), _stream()))
    return psnr, steps, status


def optimize_default_tune(B: int, max_side: int, max_T: int):
    """The launch shape the built-in table gives a batch: (threads, wgs_per_cu)."""
    out = DiskOptTune()
    _check(lib().disk_optimize_default_tune(ctypes.byref(DiskBatchMeta(B, max_side, max_T)), ctypes.byref(out)))
    return int(out.threads), int(out.wgs_per_cu)


def optimize_workspace_size(batch: Batch, tune=None):
    return int(lib().disk_optimize_workspace_size(ctypes.byref(batch.meta), None if tune is None else ctypes.byref(tune)))


def disk_basis_rotate(base, angles):
    """Angle axis: base [G0][T][3] (device) -> [G0 * len(angles)][T][3] with
    every offset rotated by each angle (radians)."""
    _dev(base, "base")
    G0, T = int(base.shape[0]), int(base.shape[1])
    G1 = len(angles)
    out = torch.empty((G0 * G1, T, 3), dtype=torch.float32, device=base.device)
    ang = (c_double * G1)(*[float(a) for a in angles])
    _check(lib().disk_basis_rotate(_ptr(base.contiguous()), G0, T, ang, G1, _ptr(out), _stream()))
    return out


DENSE_DISK, DENSE_ELLIPSE = 0, 1


def disk_dense_sv(image, pmap, kind, r0, r1, half, a0=1.0, a1=1.0, out=None):
    """Dense spatially varying convolution (the reference the sparse filter
    approximates); image [C][H][W] float32 or bfloat16, pmap [dims][H][W]."""
    _dev(image, "image")
    _dev(pmap, "pmap")
    _f32(pmap, "pmap")
    C, H, W = (int(v) for v in image.shape)
    io = BF16 if image.dtype == torch.bfloat16 else F32
    if out is None:
        out = torch.empty_like(image)
    prm = DiskDenseParams(int(kind), float(r0), float(r1), float(a0), float(a1), int(half))
    _check(lib().disk_dense_sv(ctypes.byref(prm), _ptr(image), _ptr(pmap.contiguous()), _ptr(out), C, H, W, io,
                               _stream()))
    return out


def clock_rate_khz():
    return int(lib().disk_clock_rate_khz())


def disk_fit_basis(batch: Batch, theta, scale, params: OptParams):
    """Fit the targets of ``batch`` in order by continuation (entry k starts
    from the fitted entry k-1, offsets times scale[k]); entry 0 starts from
    ``theta`` as given.  Returns (psnr_db [B], steps [B], status [B])."""
    dev = theta.device
    B = batch.B
    sc = (c_float * B)(*[float(x) for x in scale])
    psnr = torch.empty(B, dtype=torch.float32, device=dev)
    steps = torch.empty(B, dtype=torch.int32, device=dev)
    status = torch.empty(B, dtype=torch.int32, device=dev)
    L = lib()
    ws = _workspace(L.disk_fit_basis_workspace_size(ctypes.byref(batch.meta)), dev)
    _check(L.disk_fit_basis(ctypes.byref(batch.meta), _ptr(batch.desc), _ptr(batch.taps), _ptr(batch.targets),
                            _ptr(theta), _ptr(psnr), _ptr(steps), _ptr(status), sc, ctypes.byref(params.c),
                            _ptr(ws), ws.numel(), _stream()))
    return psnr, steps, status


def pack_targets(kernels, taps):
    """Lay out square kernels (odd sides) that share the layer structure
    ``taps`` as a batch: desc rows (side, L, taps_off, theta_off, target_off),
    one taps list per target, kernels concatenated."""
    taps = [int(t) for t in taps]
    T = sum(taps)
    desc, tp, flat, to = [], [], [], 0
    for b, k in enumerate(kernels):
        k = torch.as_tensor(k, dtype=torch.float32)
        desc.append((int(k.shape[0]), len(taps), len(tp), b * T, to))
        tp.extend(taps)
        flat.append(k.reshape(-1))
        to += int(k.numel())
    return (torch.tensor(desc, dtype=torch.int32), torch.tensor(tp, dtype=torch.int32), torch.cat(flat))


def fit_basis(kernels, taps, scale, params: OptParams = None):
    """Basis precompute: radial init of the first entry, then continuation
    over the entries in order.  Returns (theta [G][T][3] device, psnr_db,
    steps, status) with the per-entry results on the host."""
    params = params or OptParams(max_steps=1000, lr0=1e-2, lr1=1e-3)
    batch = make_batch(*pack_targets(kernels, taps))
    theta = disk_init_radial(batch)
    psnr, steps, status = disk_fit_basis(batch, theta, scale, params)
    return (theta.view(len(kernels), sum(int(t) for t in taps), 3), psnr.cpu().numpy(), steps.cpu().numpy(),
            status.cpu().numpy())


def disk_init_radial(batch: Batch, theta=None):
    dev = batch.desc.device
    if theta is None:
        theta = torch.empty((batch.T_total, 3), dtype=torch.float32, device=dev)
    _check(lib().disk_init_radial(ctypes.byref(batch.meta), _ptr(batch.desc), _ptr(batch.taps), _ptr(batch.targets),
                                  _ptr(theta), _stream()))
    return theta


def disk_init_shape(target, taps, seed, index=0):
    """Host FP64 shape-aware init of one target (numpy/torch CPU float32 [M][M]).
    Returns (theta float32 [T][3] CPU tensor, final radius)."""
    t = torch.as_tensor(target, dtype=torch.float32).contiguous()
    tp = torch.as_tensor([int(x) for x in taps], dtype=torch.int32).contiguous()
    T = int(tp.sum())
    out = torch.empty((T, 3), dtype=torch.float32)
    r = c_double(0.0)
    _check(lib().disk_init_shape(_ptr(t), int(t.shape[0]), int(tp.numel()), _ptr(tp), c_uint64(int(seed)),
                                 int(index), _ptr(out), ctypes.byref(r)))
    return out, r.value


def disk_init_random(target, taps, seed, index=0):
    """Host FP64 random-position init of one target.  Returns (theta float32
    [T][3] CPU tensor, extent R)."""
    t = torch.as_tensor(target, dtype=torch.float32).contiguous()
    tp = torch.as_tensor([int(x) for x in taps], dtype=torch.int32).contiguous()
    out = torch.empty((int(tp.sum()), 3), dtype=torch.float32)
    r = c_double(0.0)
    _check(lib().disk_init_random(_ptr(t), int(t.shape[0]), int(tp.numel()), _ptr(tp), c_uint64(int(seed)),
                                  int(index), _ptr(out), ctypes.byref(r)))
    return out, r.value


# ---------------------------------------------------------------------------
# learned initialiser
# ---------------------------------------------------------------------------
def disk_net_param_count():
    return int(lib().disk_net_param_count())


def net_workspace(B, device="cuda"):
    return _workspace(lib().disk_net_workspace_size(int(B)), device)


def disk_init_predict(params, targets64, half_width, ws=None):
    """Theta [B][48][3] (offsets in target pixels) for prepared inputs."""
    B = int(targets64.shape[0])
    dev = params.device
    theta = torch.empty((B, 48, 3), dtype=torch.float32, device=dev)
    L = lib()
    nws = L.disk_net_predict_workspace_size(B)
    if ws is None or ws.numel() < nws:
        ws = _workspace(nws, dev)
    _check(L.disk_init_predict(_ptr(params), _ptr(targets64), _ptr(half_width), _ptr(theta), B, _ptr(ws),
                               ws.numel(), _stream()))
    return theta


def disk_net_train_step(params, m, v, step, lr, targets64, half_width, theta_ref, ws=None, grad=None):
    """One Adam step of the initialiser on a batch; returns the loss (device
    tensor [1], before the update).  ``grad`` (optional) receives the gradient."""
    B = int(targets64.shape[0])
    dev = params.device
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    L = lib()
    nws = L.disk_net_workspace_size(B)
    if ws is None or ws.numel() < nws:
        ws = _workspace(nws, dev)
    _check(L.disk_net_train_step(_ptr(params), _ptr(m), _ptr(v), int(step), float(lr), _ptr(targets64),
                                 _ptr(half_width), _ptr(theta_ref), B, _ptr(loss), _ptr(grad), _ptr(ws), ws.numel(),
                                 _stream()))
    return loss


def disk_net_prepare_inputs(batch: Batch):
    """(targets64 int16 [B][64][64] holding BF16 bits, half_width [B])."""
    dev = batch.desc.device
    x = torch.empty((batch.B, 64, 64), dtype=torch.int16, device=dev)
    hw = torch.empty(batch.B, dtype=torch.float32, device=dev)
    _check(lib().disk_net_prepare_inputs(ctypes.byref(batch.meta), _ptr(batch.desc), _ptr(batch.targets), _ptr(x),
                                         _ptr(hw), _stream()))
    return x, hw


def disk_net_scatter_theta(batch: Batch, theta48, theta=None):
    """Write the network's [B][48][3] prediction into the batch's Theta for
    the targets of 4 layers x 12 taps.  The call leaves every other target's
    rows as they are, so when ``theta`` is None they start from the radial
    initialisation (Eq. 6), the fallback for targets the network does not
    cover."""
    if theta is None:
        theta = disk_init_radial(batch)
    _check(lib().disk_net_scatter_theta(ctypes.byref(batch.meta), _ptr(batch.desc), _ptr(batch.taps), _ptr(theta48),
                                        _ptr(theta), _stream()))
    return theta


class Captured:
    """Library calls captured once into a HIP graph (torch.cuda.CUDAGraph over
    the current device) and replayed as one launch.  ``fn`` is called once on a
    side stream to warm up, then once under capture; its return value (the
    output tensors, which live in the graph's memory pool) is kept in
    ``outputs``.  Every buffer the calls read or write must stay alive and in
    place between replays; the library's launches contain no memset or copy
    nodes, so replays recompute from the buffers' current contents."""

    def __init__(self, fn, warmup=True):
        self.graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        if warmup:
            with torch.cuda.stream(side):
                fn()
            torch.cuda.current_stream().wait_stream(side)
        with torch.cuda.graph(self.graph):
            self.outputs = fn()

    def replay(self):
        self.graph.replay()
        return self.outputs


from .autograd import DiskChain  # noqa: E402  (torch.autograd.Function over disk_forward/backward)
