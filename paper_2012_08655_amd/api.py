"""Torch-facing binding of libfoveate.so.

PyTorch supplies device memory and the current HIP stream; every step of the
computation runs in the library's HIP kernels.  Functions here only build the
C descriptors (pointers, extents, element strides) and call the C ABI.

Parameters are dicts with keys fix_x, fix_y, e0, slope, cap and optionally
block (default 32), origin_x, origin_y (default 0) and sigma_map (a CUDA
float32 tensor of nby*nbx per-fragment sigmas replacing the ramp).
"""
from __future__ import annotations

import ctypes
from typing import Mapping, Sequence

import numpy as np
import torch

from . import _native as N

_DTYPES = {torch.uint8: N.FOV_U8, torch.float32: N.FOV_F32, torch.float64: N.FOV_F64}
LAYOUTS = ("NCHW", "NHWC", "CHW", "HWC", "HW")


def _stream_handle(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def tensor_desc(t: torch.Tensor, layout: str, host: bool = False) -> N.FovTensor:
    """Describe a device tensor (or, with ``host``, a host tensor) as
    (n, c, h, w) with element strides."""
    if t.dtype not in _DTYPES:
        raise TypeError("unsupported dtype %s" % t.dtype)
    if host and t.is_cuda:
        raise ValueError("tensor must live in host memory")
    if not host and not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    s = t.stride()
    if layout == "NCHW":
        n, c, h, w = t.shape
        sn, sc, sh, sw = s
    elif layout == "NHWC":
        n, h, w, c = t.shape
        sn, sh, sw, sc = s
    elif layout == "CHW":
        c, h, w = t.shape
        n, (sc, sh, sw) = 1, s
        sn = 0
    elif layout == "HWC":
        h, w, c = t.shape
        n, (sh, sw, sc) = 1, s
        sn = 0
    elif layout == "HW":
        h, w = t.shape
        n, c, (sh, sw) = 1, 1, s
        sn = sc = 0
    else:
        raise ValueError("layout must be one of %s" % (LAYOUTS,))
    return N.FovTensor(t.data_ptr() if t.numel() else None, _DTYPES[t.dtype], n, c, h, w, sn, sc, sh, sw)


def _params_array(params, n: int):
    if isinstance(params, Mapping):
        plist = [params]
    else:
        plist = list(params)
        if len(plist) not in (1, n):
            raise ValueError("need one params dict per frame (or one shared)")
    arr = (N.FovParams * max(len(plist), 1))()
    keep = []
    for i, p in enumerate(plist):
        sm = p.get("sigma_map")
        ptr = None
        if sm is not None:
            if not (isinstance(sm, torch.Tensor) and sm.is_cuda and sm.dtype == torch.float32 and sm.is_contiguous()):
                raise TypeError("sigma_map must be a contiguous CUDA float32 tensor")
            ptr = sm.data_ptr()
            keep.append(sm)
        arr[i] = N.make_params(p, ptr)
    return arr, len(plist), keep


def _n_of(desc: N.FovTensor) -> int:
    return desc.n


def forward(x: torch.Tensor, params, out: torch.Tensor | None = None, layout: str = "NCHW",
            out_dtype: torch.dtype | None = None, stream=None) -> torch.Tensor:
    """Foveate ``x`` into ``out`` (allocated like ``x`` when None)."""
    if out is None:
        out = torch.empty_like(x, dtype=out_dtype or x.dtype)
    di, do = tensor_desc(x, layout), tensor_desc(out, layout)
    arr, npar, _keep = _params_array(params, di.n)
    N.check(N.lib().foveate_forward(ctypes.byref(di), ctypes.byref(do), arr, npar, _stream_handle(stream)))
    return out


def forward_noalloc(x: torch.Tensor, params, out: torch.Tensor, layout: str = "NCHW", stream=None) -> torch.Tensor:
    """``forward`` through the library's allocation-free entry point: the
    plan workspace is the library's fixed device array, so ``out`` must be
    given (at most 16 frames per call; calls on one GPU must not overlap)."""
    di, do = tensor_desc(x, layout), tensor_desc(out, layout)
    arr, npar, _keep = _params_array(params, di.n)
    N.check(N.lib().foveate_forward_noalloc(ctypes.byref(di), ctypes.byref(do), arr, npar, _stream_handle(stream)))
    return out


def forward_batch(frames, params, outs=None, layout: str = "HWC", out_dtype: torch.dtype | None = None,
                  stream=None):
    """Foveate a list of frames of possibly different sizes in one launch.

    ``frames`` and ``outs`` are lists of single-frame tensors in ``layout``
    ("HWC", "CHW" or "HW"); ``params`` is one dict per frame.  Returns outs.
    """
    n = len(frames)
    if len(params) != n:
        raise ValueError("need one params dict per frame")
    if outs is None:
        outs = [torch.empty_like(f, dtype=out_dtype or f.dtype) for f in frames]
    di = (N.FovTensor * max(n, 1))(*[tensor_desc(f, layout) for f in frames])
    do = (N.FovTensor * max(n, 1))(*[tensor_desc(o, layout) for o in outs])
    arr = (N.FovParams * max(n, 1))()
    keep = []
    for i, p in enumerate(params):
        a, _, k = _params_array(p, 1)
        arr[i] = a[0]
        keep.append(k)
    N.check(N.lib().foveate_forward_batch(di, do, arr, n, _stream_handle(stream)))
    return outs


def _tuning_dict(t: N.FovTuning) -> dict:
    return {"split": t.split, "strip_rows": t.strip_rows, "persistent": t.persistent, "merge": t.merge,
            "chan_split": t.chan_split, "time_us": t.time_us}


def autotune(x: torch.Tensor, params, out: torch.Tensor | None = None, layout: str = "NCHW",
             out_dtype: torch.dtype | None = None, reps: int = 5, stream=None) -> dict:
    """Time every launch configuration on this call and cache the fastest for
    its workload class (later forward calls of the class use it).  ``out``
    holds the foveated result on return.  Returns the chosen configuration."""
    if out is None:
        out = torch.empty_like(x, dtype=out_dtype or x.dtype)
    di, do = tensor_desc(x, layout), tensor_desc(out, layout)
    arr, npar, _keep = _params_array(params, di.n)
    t = N.FovTuning()
    N.check(N.lib().foveate_autotune(ctypes.byref(di), ctypes.byref(do), arr, npar, int(reps),
                                     _stream_handle(stream), ctypes.byref(t)))
    return _tuning_dict(t)


def autotune_batch(frames, params, outs, layout: str = "HWC", reps: int = 5, stream=None) -> dict:
    """As ``autotune`` for a ``forward_batch`` call."""
    n = len(frames)
    di = (N.FovTensor * max(n, 1))(*[tensor_desc(f, layout) for f in frames])
    do = (N.FovTensor * max(n, 1))(*[tensor_desc(o, layout) for o in outs])
    arr = (N.FovParams * max(n, 1))()
    keep = []
    for i, p in enumerate(params):
        a, _, k = _params_array(p, 1)
        arr[i] = a[0]
        keep.append(k)
    t = N.FovTuning()
    N.check(N.lib().foveate_autotune_batch(di, do, arr, n, int(reps), _stream_handle(stream), ctypes.byref(t)))
    return _tuning_dict(t)


def tuning_force(split: int | None = None, strip_rows: int = 64, persistent: int = 0, merge: int = 0,
                 chan_split: int = 0):
    """Force a launch configuration for this thread's forward calls
    (``split=None`` returns to the cache and defaults)."""
    if split is None:
        N.check(N.lib().foveate_tuning_force(None))
        return
    t = N.FovTuning(int(split), int(strip_rows), int(persistent), int(merge), int(chan_split), 0.0)
    N.check(N.lib().foveate_tuning_force(ctypes.byref(t)))


def tuning_clear():
    N.check(N.lib().foveate_tuning_clear())


def tuning_count() -> int:
    n = ctypes.c_int32()
    N.check(N.lib().foveate_tuning_count(ctypes.byref(n)))
    return n.value


def tuning_save(path: str):
    N.check(N.lib().foveate_tuning_save(str(path).encode()))


def tuning_load(path: str):
    N.check(N.lib().foveate_tuning_load(str(path).encode()))


def backward(grad_out: torch.Tensor, params, grad_in: torch.Tensor | None = None, layout: str = "NCHW",
             stream=None) -> torch.Tensor:
    """grad_in = A^T grad_out for the same parameters as the forward."""
    if grad_in is None:
        grad_in = torch.empty_like(grad_out)
    dg, di = tensor_desc(grad_out, layout), tensor_desc(grad_in, layout)
    arr, npar, _keep = _params_array(params, dg.n)
    N.check(N.lib().foveate_backward(ctypes.byref(dg), ctypes.byref(di), arr, npar, _stream_handle(stream)))
    return grad_in


def profile_begin(capacity: int, every: int = 1):
    """Start recording main-kernel durations of this thread's forward calls
    (one call in ``every``)."""
    N.check(N.lib().foveate_profile_begin(int(capacity)))
    if every != 1:
        N.check(N.lib().foveate_profile_every(int(every)))


def profile_end(capacity: int) -> np.ndarray:
    """Wait for and return the recorded main-kernel durations (ms)."""
    buf = (ctypes.c_float * max(int(capacity), 1))()
    cnt = ctypes.c_int32()
    N.check(N.lib().foveate_profile_end(buf, int(capacity), ctypes.byref(cnt)))
    return np.array(buf[:cnt.value], dtype=np.float64)


def grid(h: int, w: int, params: Mapping) -> tuple[int, int]:
    """(nby, nbx) fragment rows/columns of an h x w frame."""
    p = N.make_params(params)
    nbx, nby = ctypes.c_int32(), ctypes.c_int32()
    N.check(N.lib().foveate_grid(h, w, ctypes.byref(p), ctypes.byref(nbx), ctypes.byref(nby)))
    return nby.value, nbx.value


def csf_params(h: int, w: int, params: Mapping, e_corner: float, f_max: float = 0.0, cap: float = 1e6) -> dict:
    """Copy of ``params`` whose ramp (e0, slope, cap) is the Geisler-Perry
    blur model for an h x w frame whose corner sits at ``e_corner`` degrees
    (foveate_csf_params)."""
    p = N.make_params(params)
    N.check(N.lib().foveate_csf_params(int(h), int(w), float(e_corner), float(f_max), float(cap), ctypes.byref(p)))
    out = dict(params)
    out["e0"], out["slope"], out["cap"] = p.e0, p.slope, p.cap
    return out


def fragment_shift(params: Mapping) -> dict:
    """Copy of ``params`` with the tiling origin that centres one fragment on
    the fixation (foveate_fragment_shift)."""
    ox, oy = ctypes.c_int32(), ctypes.c_int32()
    N.check(N.lib().foveate_fragment_shift(float(params["fix_x"]), float(params["fix_y"]),
                                           int(params.get("block", 32)), ctypes.byref(ox), ctypes.byref(oy)))
    out = dict(params)
    out["origin_x"], out["origin_y"] = ox.value, oy.value
    return out


def plan_device(h: int, w: int, params: Mapping, device="cuda"):
    """Per-fragment (sigma f64, radius i32) computed by the device planner."""
    nby, nbx = grid(h, w, params)
    sig = torch.empty((nby, nbx), dtype=torch.float64, device=device)
    rad = torch.empty((nby, nbx), dtype=torch.int32, device=device)
    arr, _, _keep = _params_array(params, 1)
    N.check(N.lib().foveate_plan(h, w, arr, ctypes.c_void_p(sig.data_ptr()), ctypes.c_void_p(rad.data_ptr()),
                                 _stream_handle()))
    return sig, rad


def plan_host(h: int, w: int, params: Mapping):
    """Per-fragment (sigma, radius) computed by the host planner."""
    nby, nbx = grid(h, w, params)
    sig = np.zeros((nby, nbx), np.float64)
    rad = np.zeros((nby, nbx), np.int32)
    p = N.make_params(params)
    N.check(N.lib().foveate_plan_host(h, w, ctypes.byref(p), ctypes.c_void_p(sig.ctypes.data),
                                      ctypes.c_void_p(rad.ctypes.data)))
    return sig, rad


class FoveateFn(torch.autograd.Function):
    """y = A_p x with the hand-written adjoint as its backward.  Gradients flow
    to x only: sigma and r = ceil(3 sigma) are piecewise constant in the
    parameters."""

    @staticmethod
    def forward(ctx, x, params, layout):
        ctx.params = params
        ctx.layout = layout
        return forward(x, params, layout=layout)

    @staticmethod
    def backward(ctx, g):
        g = g.contiguous()
        return backward(g, ctx.params, layout=ctx.layout), None, None


def foveate(x: torch.Tensor, params, layout: str = "NCHW") -> torch.Tensor:
    """Differentiable foveation of a float tensor (f32 or f64)."""
    return FoveateFn.apply(x, params, layout)
