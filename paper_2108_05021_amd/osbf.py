"""Thin Python binding of the C ABI in ``include/osbf.h`` (ctypes).

Argument marshalling only: every step of the filter runs in the HIP kernels of
``libosbf.so``.  PyTorch provides device memory (the caching allocator) and the
current stream.  If the library is missing the calls raise; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libosbf.so")

SUCCESS = 0
DTYPES = {torch.float32: 0, torch.float16: 1, torch.bfloat16: 2}
WINDOWS = ("R", "L", "D", "U", "SE", "SW", "NE", "NW")
MAX_RADIUS = 32

_lib = None


class Image(ctypes.Structure):
    """osbf_image: one image of a batch (strides in elements, 0 = contiguous)."""
    _fields_ = [("src", ctypes.c_void_p), ("dst", ctypes.c_void_p), ("planes", ctypes.c_int32),
                ("height", ctypes.c_int32), ("width", ctypes.c_int32), ("radius", ctypes.c_int32),
                ("iterations", ctypes.c_int32), ("src_plane_stride", ctypes.c_int64),
                ("src_row_stride", ctypes.c_int64), ("dst_plane_stride", ctypes.c_int64),
                ("dst_row_stride", ctypes.c_int64)]


class Batch(ctypes.Structure):
    """osbf_batch: a prepared batch (plain data)."""
    _fields_ = [("n", ctypes.c_int32), ("dtype", ctypes.c_int32), ("rounds", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("max_items", ctypes.c_int64), ("total_items", ctypes.c_int64),
                ("ws", ctypes.c_void_p), ("descs_off", ctypes.c_size_t), ("items_off", ctypes.c_size_t),
                ("counts_off", ctypes.c_size_t), ("identity", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 7)]


class OsbfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"osbf status {status}: {msg}")
        self.status = status


def lib():
    """Load ``libosbf.so`` (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2108_05021_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    vp, sz, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32
    L.osbf_abi_version.argtypes = []
    L.osbf_abi_version.restype = i32
    L.osbf_status_string.argtypes = [ctypes.c_int]
    L.osbf_status_string.restype = ctypes.c_char_p
    L.osbf_last_error.argtypes = []
    L.osbf_last_error.restype = ctypes.c_char_p
    L.osbf_forward_workspace_size.argtypes = [i32, i32, i32, ctypes.c_int, i32, i32]
    L.osbf_forward_workspace_size.restype = sz
    L.osbf_forward.argtypes = [vp, vp, i32, i32, i32, ctypes.c_int, i32, i32, ctypes.c_int,
                               vp, vp, i32, vp, sz, vp]
    L.osbf_forward.restype = ctypes.c_int
    L.osbf_forward_noalloc.argtypes = [vp, vp, i32, i32, i32, ctypes.c_int, i32, i32, ctypes.c_int, vp]
    L.osbf_forward_noalloc.restype = ctypes.c_int
    L.osbf_forward_fast.argtypes = [vp, vp, i32, i32, i32, ctypes.c_int, i32, i32, ctypes.c_int, vp, sz, vp]
    L.osbf_forward_fast.restype = ctypes.c_int
    L.osbf_box_forward.argtypes = [vp, vp, i32, i32, i32, ctypes.c_int, i32, i32, ctypes.c_int, vp, sz, vp]
    L.osbf_box_forward.restype = ctypes.c_int
    L.osbf_backward_workspace_size.argtypes = [i32, i32, i32, i32, i32, i32]
    L.osbf_backward_workspace_size.restype = sz
    L.osbf_backward.argtypes = [vp, vp, i32, i32, i32, i32, i32, ctypes.c_int, vp, vp, i32, vp, sz, vp]
    L.osbf_backward.restype = ctypes.c_int
    L.osbf_batched_workspace_size.argtypes = [ctypes.POINTER(Image), i32, ctypes.c_int]
    L.osbf_batched_workspace_size.restype = sz
    L.osbf_batched_prepare.argtypes = [ctypes.POINTER(Image), i32, ctypes.c_int, ctypes.c_int, vp, sz,
                                       ctypes.POINTER(Batch), vp]
    L.osbf_batched_prepare.restype = ctypes.c_int
    L.osbf_batched_launch.argtypes = [ctypes.POINTER(Batch), vp]
    L.osbf_batched_launch.restype = ctypes.c_int
    L.osbf_batched.argtypes = [ctypes.POINTER(Image), i32, ctypes.c_int, ctypes.c_int, vp, sz, vp]
    L.osbf_batched.restype = ctypes.c_int
    L.osbf_forward_plan.argtypes = [i32, i32, i32, ctypes.c_int, i32, i32, i32] + [ctypes.POINTER(i32)] * 4
    L.osbf_forward_plan.restype = ctypes.c_int
    L.osbf3d_forward_workspace_size.argtypes = [i32, i32, i32, i32, i32, i32]
    L.osbf3d_forward_workspace_size.restype = sz
    L.osbf3d_forward.argtypes = [vp, vp, i32, i32, i32, i32, i32, i32, vp, vp, sz, vp]
    L.osbf3d_forward.restype = ctypes.c_int
    L.osbf_gaussian_workspace_size.argtypes = [i32, i32, i32, i32, i32]
    L.osbf_gaussian_workspace_size.restype = sz
    L.osbf_gaussian_forward.argtypes = [vp, vp, i32, i32, i32, i32, ctypes.c_float, i32, vp, vp, sz, vp]
    L.osbf_gaussian_forward.restype = ctypes.c_int
    L.osbf_autotune.argtypes = [vp, vp, i32, i32, i32, ctypes.c_int, i32, i32, vp] + [ctypes.POINTER(i32)] * 3
    L.osbf_autotune.restype = ctypes.c_int
    L.osbf_batched_autotune_workspace_size.argtypes = [ctypes.POINTER(Image), i32, ctypes.c_int]
    L.osbf_batched_autotune_workspace_size.restype = sz
    L.osbf_batched_autotune.argtypes = [ctypes.POINTER(Image), i32, ctypes.c_int, vp, sz, vp,
                                        ctypes.POINTER(i32)]
    L.osbf_batched_autotune.restype = ctypes.c_int
    L.osbf_autotune_clear.argtypes = []
    L.osbf_autotune_clear.restype = None
    _lib = L
    return L


def _check(status: int):
    if status != SUCCESS:
        raise OsbfError(status, lib().osbf_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _geometry(x: torch.Tensor):
    if x.dim() < 2:
        raise ValueError("expected (..., H, W)")
    if not x.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    H, W = x.shape[-2], x.shape[-1]
    planes = x.numel() // (H * W) if H * W else 0
    return planes, H, W


def _strided_geometry(x: torch.Tensor):
    """(planes, H, W, plane stride, row stride) of a (..., H, W) tensor whose
    rows are contiguous and whose leading dimensions collapse into one plane
    index with a uniform stride (crops and other views of larger tensors);
    strides in elements, 0 where a single plane or row makes them moot."""
    if x.dim() < 2:
        raise ValueError("expected (..., H, W)")
    H, W = x.shape[-2], x.shape[-1]
    st = x.stride()
    if W > 1 and st[-1] != 1:
        raise ValueError("expected rows with unit stride along W")
    ld = st[-2] if H > 1 else 0
    if H > 1 and ld < W:
        raise ValueError(f"rows overlap (row stride {ld} < width {W})")
    planes = x.numel() // (H * W) if H * W else 0
    ps = 0
    lead = [(n, s) for n, s in zip(x.shape[:-2], st[:-2]) if n != 1]
    if planes > 1:
        ps = lead[-1][1]
        expect = ps
        for n, s in reversed(lead):
            if s != expect:
                raise ValueError("leading dimensions must collapse into one plane index with a uniform stride")
            expect = s * n
        if ps < H * max(ld, W):
            raise ValueError(f"planes overlap (plane stride {ps} < height x row stride)")
    return planes, H, W, ps, ld


def forward_workspace_size(planes, H, W, dtype, r, T) -> int:
    return int(lib().osbf_forward_workspace_size(planes, H, W, DTYPES[dtype], r, T))


def forward_plan(planes, H, W, dtype, r, T, ck: int = 0) -> dict:
    """Launch plan of osbf_forward: tile shape, fused sweeps, launches."""
    v = [ctypes.c_int32() for _ in range(4)]
    _check(lib().osbf_forward_plan(planes, H, W, DTYPES[dtype], r, T, ck, *[ctypes.byref(t) for t in v]))
    return {"tile": (v[0].value, v[1].value), "fused": v[2].value, "launches": v[3].value}


def osbf_forward(src, dst, r: int, T: int, *, sel=None, ckpt=None, ck: int = 0, ws=None):
    """Direct call of the C entry point on preallocated tensors."""
    planes, H, W = _geometry(src)
    status = lib().osbf_forward(
        _ptr(src), _ptr(dst), planes, H, W, DTYPES[src.dtype], r, T, 0,
        _ptr(sel), _ptr(ckpt), ck, _ptr(ws), 0 if ws is None else ws.numel() * ws.element_size(),
        _stream(src.device))
    _check(status)


def forward(x: torch.Tensor, r: int, T: int, *, return_sel: bool = False,
            ckpt_every: int = 0, out: torch.Tensor | None = None):
    """T sweeps of the one-sided box filter on a (..., H, W) device tensor.

    Returns the filtered tensor (same shape and dtype); with ``return_sel``
    also the uint8 selection maps [T, *x.shape]; with ``ckpt_every`` > 0 also
    the checkpoints [ceil(T/ckpt_every), *x.shape] of U^0, U^ck, ...
    """
    planes, H, W = _geometry(x)
    y = torch.empty_like(x) if out is None else out
    sel = torch.empty((T, *x.shape), dtype=torch.uint8, device=x.device) if return_sel else None
    ckpt = None
    if ckpt_every > 0:
        nck = (T + ckpt_every - 1) // ckpt_every
        ckpt = torch.empty((nck, *x.shape), dtype=x.dtype, device=x.device)
    nbytes = forward_workspace_size(planes, H, W, x.dtype, r, T)
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=x.device) if nbytes else None
    osbf_forward(x, y, r, T, sel=sel, ckpt=ckpt, ck=ckpt_every, ws=ws)
    res = [y]
    if return_sel:
        res.append(sel)
    if ckpt is not None:
        res.append(ckpt)
    return res[0] if len(res) == 1 else tuple(res)


def forward_noalloc(x: torch.Tensor, r: int, T: int, *, out: torch.Tensor | None = None):
    """T sweeps through osbf_forward_noalloc: no workspace argument, the
    library's per-device scratch holds the ping-pong iterate (images up to
    OSBF_NOALLOC_SCRATCH_BYTES)."""
    planes, H, W = _geometry(x)
    y = torch.empty_like(x) if out is None else out
    _check(lib().osbf_forward_noalloc(_ptr(x), _ptr(y), planes, H, W, DTYPES[x.dtype], r, T, 0,
                                      _stream(x.device)))
    return y


NOALLOC_SCRATCH_BYTES = 64 << 20


def backward_workspace_size(planes, H, W, r, T, ck: int = 0) -> int:
    return int(lib().osbf_backward_workspace_size(planes, H, W, r, T, ck))


def osbf_backward(grad_out, grad_in, r: int, T: int, *, sel=None, ckpt=None, ck: int = 0, ws=None):
    """Direct call of the C entry point on preallocated FP32 tensors."""
    # the C entry point takes FP32 gradients and checkpoints and uint8 maps
    for name, t, dt in (("grad_out", grad_out, torch.float32), ("grad_in", grad_in, torch.float32),
                        ("ckpt", ckpt, torch.float32), ("sel", sel, torch.uint8)):
        if t is not None and t.dtype != dt:
            raise TypeError(f"osbf_backward: {name} must be {dt}, got {t.dtype}")
    planes, H, W = _geometry(grad_out)
    status = lib().osbf_backward(
        _ptr(grad_out), _ptr(grad_in), planes, H, W, r, T, 0, _ptr(sel), _ptr(ckpt), ck,
        _ptr(ws), 0 if ws is None else ws.numel() * ws.element_size(), _stream(grad_out.device))
    _check(status)


def backward(grad_out: torch.Tensor, r: int, T: int, *, sel=None, ckpt=None, ck: int = 0):
    """Gradient w.r.t. the input of T sweeps, given the forward's selection
    maps ``sel`` [T, ...] or its checkpoints ``ckpt`` taken every ``ck`` sweeps."""
    planes, H, W = _geometry(grad_out)
    grad_in = torch.empty_like(grad_out)
    n = backward_workspace_size(planes, H, W, r, T, ck if ckpt is not None else 0)
    ws = torch.empty(max(n, 1), dtype=torch.uint8, device=grad_out.device) if n else None
    osbf_backward(grad_out, grad_in, r, T, sel=sel, ckpt=ckpt, ck=ck, ws=ws)
    return grad_in


class OSBFFunction(torch.autograd.Function):
    """Differentiable one-sided box filter (FP32).  The backward holds every
    selection at its forward value; ``ckpt_every`` > 0 stores iterates every
    that many sweeps instead of all T uint8 selection maps."""

    @staticmethod
    def forward(ctx, x, r: int, T: int, ckpt_every: int = 0):
        if x.dtype != torch.float32:
            # the backward entry point reads FP32 checkpoints; 16-bit storage
            # has no gradient path
            raise TypeError(f"OSBFFunction: input must be torch.float32, got {x.dtype}")
        x = x.contiguous()
        if ckpt_every > 0:
            y, ck = forward(x, r, T, ckpt_every=ckpt_every)
            ctx.save_for_backward(ck)
            ctx.mode = "ckpt"
        else:
            y, sel = forward(x, r, T, return_sel=True)
            ctx.save_for_backward(sel)
            ctx.mode = "sel"
        ctx.r, ctx.T, ctx.ck = r, T, ckpt_every
        return y

    @staticmethod
    def backward(ctx, gy):
        (saved,) = ctx.saved_tensors
        gy = gy.contiguous().float()
        if ctx.mode == "ckpt":
            gx = backward(gy, ctx.r, ctx.T, ckpt=saved, ck=ctx.ck)
        else:
            gx = backward(gy, ctx.r, ctx.T, sel=saved)
        return gx, None, None, None


def osbf(x: torch.Tensor, r: int, T: int, ckpt_every: int = 0) -> torch.Tensor:
    """The filter as a differentiable op (see OSBFFunction)."""
    return OSBFFunction.apply(x, r, T, ckpt_every)


def _images(xs, outs, radii, iters):
    """The osbf_image list of a batch.  Every image and output must share the
    first image's dtype and device (the C ABI carries one dtype for the whole
    batch), each output must match its input's shape, and there must be one
    radius and one iteration count per image.  Images and outputs may be
    strided views (rows contiguous): their strides go into the image list."""
    xs, outs, radii, iters = list(xs), list(outs), list(radii), list(iters)
    if not (len(xs) == len(outs) == len(radii) == len(iters)):
        raise ValueError(f"batch lists differ in length: {len(xs)} images, {len(outs)} outputs, "
                         f"{len(radii)} radii, {len(iters)} iteration counts")
    if xs:
        dt, dev = xs[0].dtype, xs[0].device
        for i, (x, y) in enumerate(zip(xs, outs)):
            if x.dtype != dt or y.dtype != dt:
                raise ValueError(f"image {i}: dtype {x.dtype} / output {y.dtype}, batch dtype is {dt}")
            if x.device != dev or y.device != dev:
                raise ValueError(f"image {i}: not on {dev}")
            if y.shape != x.shape:
                raise ValueError(f"image {i}: output shape {tuple(y.shape)} != input shape {tuple(x.shape)}")
    arr = (Image * len(xs))()
    for i, (x, y, r, T) in enumerate(zip(xs, outs, radii, iters)):
        planes, H, W, sps, sld = _strided_geometry(x)
        _, _, _, dps, dld = _strided_geometry(y)
        arr[i] = Image(x.data_ptr(), y.data_ptr(), planes, H, W, int(r), int(T), sps, sld, dps, dld)
    return arr


class BatchPlan:
    """A prepared batch: per-image outputs, workspace and tables on the device.
    ``launch()`` only enqueues kernels, so it can be captured in a CUDA/HIP
    graph and replayed (each replay recomputes the outputs from the inputs)."""

    def __init__(self, xs, radii, iters, outs=None):
        if not xs:
            raise ValueError("empty batch")
        self.xs = list(xs)
        self.outs = [torch.empty(x.shape, dtype=x.dtype, device=x.device) for x in xs] if outs is None \
            else list(outs)
        dt = DTYPES[xs[0].dtype]
        self.images = _images(self.xs, self.outs, radii, iters)
        n = lib().osbf_batched_workspace_size(self.images, len(xs), dt)
        if n == ctypes.c_size_t(-1).value:   # invalid: let prepare report the status
            _check(lib().osbf_batched_prepare(self.images, len(xs), dt, 0, None, 0,
                                              ctypes.byref(Batch()), _stream(xs[0].device)))
        self.ws = torch.empty(max(n, 1), dtype=torch.uint8, device=xs[0].device)
        self.batch = Batch()
        _check(lib().osbf_batched_prepare(self.images, len(xs), dt, 0, _ptr(self.ws), n,
                                          ctypes.byref(self.batch), _stream(xs[0].device)))

    def launch(self):
        _check(lib().osbf_batched_launch(ctypes.byref(self.batch), _stream(self.xs[0].device)))
        return self.outs


def batched(xs, radii, iters, outs=None):
    """Filter a list of (..., H, W) device tensors of one dtype, each with its
    own radius and iteration count, in one batched call."""
    outs = [torch.empty(x.shape, dtype=x.dtype, device=x.device) for x in xs] if outs is None else list(outs)
    dt = DTYPES[xs[0].dtype]
    imgs = _images(xs, outs, radii, iters)
    n = lib().osbf_batched_workspace_size(imgs, len(xs), dt)
    if n == ctypes.c_size_t(-1).value:   # invalid: let the call report the status
        _check(lib().osbf_batched(imgs, len(xs), dt, 0, None, 0, _stream(xs[0].device)))
    ws = torch.empty(max(n, 1), dtype=torch.uint8, device=xs[0].device)
    _check(lib().osbf_batched(imgs, len(xs), dt, 0, _ptr(ws), n, _stream(xs[0].device)))
    return outs


def _mode_forward(fn, x, r, T, out):
    planes, H, W = _geometry(x)
    y = torch.empty_like(x) if out is None else out
    nbytes = forward_workspace_size(planes, H, W, x.dtype, r, T)
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=x.device) if nbytes else None
    _check(fn(_ptr(x), _ptr(y), planes, H, W, DTYPES[x.dtype], r, T, 0, _ptr(ws),
              0 if ws is None else ws.numel(), _stream(x.device)))
    return y


def forward_fast(x: torch.Tensor, r: int, T: int, *, out: torch.Tensor | None = None):
    """T sweeps of the fast approximation (Alg. 3) on a (..., H, W) tensor."""
    return _mode_forward(lib().osbf_forward_fast, x, r, T, out)


def box_forward(x: torch.Tensor, r: int, T: int, *, out: torch.Tensor | None = None):
    """T sweeps of the classical (2r+1)^2 box filter (replicate boundary)."""
    return _mode_forward(lib().osbf_box_forward, x, r, T, out)


def forward3d(x: torch.Tensor, r: int, T: int, *, return_sel: bool = False,
              out: torch.Tensor | None = None):
    """T sweeps of the volume filter (14 windows) on a (..., D, H, W) FP32
    device tensor; with ``return_sel`` also the uint8 maps [T, *x.shape]."""
    if x.dim() < 3:
        raise ValueError("expected (..., D, H, W)")
    if not x.is_contiguous() or x.dtype != torch.float32:
        raise ValueError("expected a contiguous float32 tensor")
    D, H, W = x.shape[-3:]
    vols = x.numel() // (D * H * W) if D * H * W else 0
    y = torch.empty_like(x) if out is None else out
    sel = torch.empty((T, *x.shape), dtype=torch.uint8, device=x.device) if return_sel else None
    n = int(lib().osbf3d_forward_workspace_size(vols, D, H, W, r, T))
    if n == (1 << 64) - 1:
        n = 0  # invalid arguments: the entry point reports the error
    ws = torch.empty(max(n, 1), dtype=torch.uint8, device=x.device) if n else None
    _check(lib().osbf3d_forward(_ptr(x), _ptr(y), vols, D, H, W, r, T, _ptr(sel), _ptr(ws),
                                0 if ws is None else ws.numel(), _stream(x.device)))
    return (y, sel) if return_sel else y


def gaussian_forward(x: torch.Tensor, r: int, sigma: float, T: int, *, return_sel: bool = False,
                     out: torch.Tensor | None = None):
    """T sweeps of the one-sided Gaussian filter (weights exp(-u^2/(2 sigma^2))
    per axis, the box filter's eight windows) on a (..., H, W) FP32 tensor."""
    if x.dtype != torch.float32:
        raise ValueError("expected a float32 tensor")
    planes, H, W = _geometry(x)
    y = torch.empty_like(x) if out is None else out
    sel = torch.empty((T, *x.shape), dtype=torch.uint8, device=x.device) if return_sel else None
    n = int(lib().osbf_gaussian_workspace_size(planes, H, W, r, T))
    if n == (1 << 64) - 1:
        n = 0  # invalid arguments: the entry point reports the error
    ws = torch.empty(max(n, 1), dtype=torch.uint8, device=x.device) if n else None
    _check(lib().osbf_gaussian_forward(_ptr(x), _ptr(y), planes, H, W, r, float(sigma), T, _ptr(sel),
                                       _ptr(ws), 0 if ws is None else ws.numel(), _stream(x.device)))
    return (y, sel) if return_sel else y


def autotune(x: torch.Tensor, r: int, T: int) -> dict:
    """Measure osbf_forward's launch plans on x's shape and dtype (x is read,
    a scratch output is written) and keep the fastest for this device and
    problem class; returns the chosen tile and fused sweeps.  Blocks."""
    planes, H, W = _geometry(x)
    scratch = torch.empty_like(x)
    tw, th, k = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().osbf_autotune(_ptr(x), _ptr(scratch), planes, H, W, DTYPES[x.dtype], r, T,
                               _stream(x.device), ctypes.byref(tw), ctypes.byref(th), ctypes.byref(k)))
    return {"tile": (tw.value, th.value), "fused": k.value}


def batched_autotune(xs, radii, iters) -> dict:
    """Tune the rows per batched work item for the radii of this batch
    (osbf_batched_autotune); returns {radius: rows}.  The batch's outputs are
    scratch during tuning."""
    outs = [torch.empty(x.shape, dtype=x.dtype, device=x.device) for x in xs]
    dt = DTYPES[xs[0].dtype]
    imgs = _images(xs, outs, radii, iters)
    n = lib().osbf_batched_autotune_workspace_size(imgs, len(xs), dt)
    if n == ctypes.c_size_t(-1).value:
        _check(lib().osbf_batched_autotune(imgs, len(xs), dt, None, 0, _stream(xs[0].device), None))
    ws = torch.empty(max(n, 1), dtype=torch.uint8, device=xs[0].device)
    rows = (ctypes.c_int32 * (MAX_RADIUS + 1))()
    _check(lib().osbf_batched_autotune(imgs, len(xs), dt, _ptr(ws), n, _stream(xs[0].device), rows))
    return {r: rows[r] for r in range(MAX_RADIUS + 1) if rows[r]}


def autotune_clear() -> None:
    """Forget every autotuned plan."""
    lib().osbf_autotune_clear()
