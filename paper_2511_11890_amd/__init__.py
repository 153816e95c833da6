"""Harpia-style chunked volumetric filters for MI355X (gfx950).

Python layer over libharpia (include/harpia.h).  Volumes are [nz, ny, nx]
arrays: CUDA/HIP torch tensors run resident on the current torch stream;
CPU torch tensors and numpy arrays run through the library's chunk engine
(copied to the GPU chunk by chunk under a device-memory budget).  All
filtering happens in the HIP library; this package only marshals arguments
and allocates outputs.
"""
from __future__ import annotations

import numpy as np

from . import _lib
from ._lib import HarpiaError, harpia_plan, harpia_stats

__all__ = ["gaussian", "mean", "unsharp", "edge", "hessian", "local_threshold", "otsu", "erode", "dilate", "erode_dilate", "opening", "closing", "morph",
           "plan", "gauss_radius", "version", "HarpiaError", "harpia_stats", "Exec",
           "gaussian_backward", "morph_backward", "GaussianFn", "MorphFn", "GaussDilateFn",
           "gaussian_batched", "morph_batched", "GaussDilateBatch", "autotune_gaussian",
           "autotune_erode_dilate", "tune_clear", "tune_entries", "tune_save", "tune_load"]


def _torch():
    import torch
    return torch


_NP_DT = {np.dtype(np.uint8): _lib.HARPIA_U8, np.dtype(np.uint16): _lib.HARPIA_U16,
          np.dtype(np.float32): _lib.HARPIA_F32, np.dtype(np.float16): _lib.HARPIA_F16}
_DT_NP = {v: k for k, v in _NP_DT.items()}


def _torch_dt():
    t = _torch()
    return {t.uint8: _lib.HARPIA_U8, t.uint16: _lib.HARPIA_U16, t.float32: _lib.HARPIA_F32,
            t.float16: _lib.HARPIA_F16, t.bfloat16: _lib.HARPIA_BF16}


_NAMES = {"u8": _lib.HARPIA_U8, "u16": _lib.HARPIA_U16, "f32": _lib.HARPIA_F32,
          "f16": _lib.HARPIA_F16, "bf16": _lib.HARPIA_BF16}


class Exec:
    """Execution options (harpia_exec): device budget in bytes (0: fraction of
    free memory), budget fraction, chunk extent {z, y, x} (zeros: z-slabs),
    flags, and an optional harpia_stats to fill."""

    def __init__(self, budget: int = 0, fraction: float = 0.0, chunk=(0, 0, 0),
                 force_chunked: bool = False, stats: harpia_stats | None = None):
        self.budget = budget
        self.fraction = fraction
        self.chunk = tuple(chunk)
        self.force_chunked = force_chunked
        self.stats = stats


def version() -> str:
    return _lib.load().harpia_version().decode()


def gauss_radius(sigma: float, truncate: float = 3.0) -> int:
    return int(_lib.load().harpia_gauss_radius(float(sigma), float(truncate)))


def _is_torch(x) -> bool:
    try:
        torch = _torch()
    except ImportError:  # pragma: no cover
        return False
    return isinstance(x, torch.Tensor)


def _dtype_code(x) -> int:
    if _is_torch(x):
        try:
            return _torch_dt()[x.dtype]
        except KeyError:
            raise HarpiaError(_lib.HARPIA_ERR_DTYPE, "unsupported dtype %s" % x.dtype)
    try:
        return _NP_DT[np.asarray(x).dtype]
    except KeyError:
        raise HarpiaError(_lib.HARPIA_ERR_DTYPE, "unsupported dtype %s" % np.asarray(x).dtype)


def _check_volume(x):
    if x.ndim != 3:
        raise ValueError("volumes are 3D [nz, ny, nx]")
    if _is_torch(x):
        if not x.is_contiguous():
            raise ValueError("volume must be contiguous")
    elif not x.flags["C_CONTIGUOUS"]:
        raise ValueError("volume must be C-contiguous")


def _empty_like(x, code: int):
    if _is_torch(x):
        torch = _torch()
        inv = {v: k for k, v in _torch_dt().items()}
        return torch.empty(tuple(x.shape), dtype=inv[code], device=x.device,
                           pin_memory=(x.device.type == "cpu" and x.is_pinned()))
    if code not in _DT_NP:
        raise HarpiaError(_lib.HARPIA_ERR_DTYPE, "numpy has no bfloat16")
    return np.empty(x.shape, dtype=_DT_NP[code])


def _ptr(x) -> int:
    return x.data_ptr() if _is_torch(x) else x.ctypes.data


def _exec(x, ex: Exec | None, flags: int = 0):
    stream = None
    if _is_torch(x) and x.is_cuda:
        torch = _torch()
        stream = torch.cuda.current_stream(x.device).cuda_stream
    ex = ex or Exec()
    if ex.force_chunked:
        flags |= _lib.HARPIA_F_FORCE_CHUNKED
    return _lib.make_exec(ex.budget, ex.fraction, ex.chunk, stream, flags, ex.stats)


def _device_guard(x):
    if _is_torch(x) and x.is_cuda:
        return _torch().cuda.device(x.device)
    import contextlib
    return contextlib.nullcontext()


def _triple(v, cast):
    if np.ndim(v) == 0:
        return (cast(v),) * 3
    v = tuple(cast(t) for t in v)
    if len(v) != 3:
        raise ValueError("expected a scalar or a (z, y, x) triple")
    return v


def _code(dt) -> int:
    if dt is None:
        return -1
    if isinstance(dt, str):
        return _NAMES[dt]
    if _is_torch_dtype(dt):
        return _torch_dt()[dt]
    return _NP_DT[np.dtype(dt)]


def _is_torch_dtype(dt) -> bool:
    try:
        return isinstance(dt, _torch().dtype)
    except ImportError:  # pragma: no cover
        return False


def gaussian(x, sigma, truncate: float = 3.0, out=None, out_dtype=None, ex: Exec | None = None):
    """Gaussian smoothing (reflect boundary, FP64 taps, FP32 accumulation).
    out dtype: float32 for u8/u16/f32 inputs, the input's dtype for f16/bf16
    unless out_dtype says float32."""
    _check_volume(x)
    ic = _dtype_code(x)
    oc = _code(out_dtype)
    if oc < 0:
        oc = ic if ic in (_lib.HARPIA_F16, _lib.HARPIA_BF16) else _lib.HARPIA_F32
    if out is None:
        out = _empty_like(x, oc)
    else:
        _check_volume(out)
        oc = _dtype_code(out)
    e = _exec(x, ex)
    with _device_guard(x):
        _lib.check(_lib.load().harpia_gaussian3d(
            _ptr(x), ic, _ptr(out), oc, _lib.i64_3(x.shape), _lib.f64_3(_triple(sigma, float)),
            float(truncate), _lib.HARPIA_BORDER_REFLECT, e))
    return out


def _smooth_out(x, out, out_dtype):
    _check_volume(x)
    ic = _dtype_code(x)
    oc = _code(out_dtype)
    if oc < 0:
        oc = ic if ic in (_lib.HARPIA_F16, _lib.HARPIA_BF16) else _lib.HARPIA_F32
    if out is None:
        out = _empty_like(x, oc)
    else:
        _check_volume(out)
        oc = _dtype_code(out)
    return ic, oc, out


def mean(x, radius=1, out=None, out_dtype=None, ex: Exec | None = None):
    """Mean (box) filter: average over the (2r+1)-box per axis, reflect
    boundary; output dtypes as for gaussian()."""
    ic, oc, out = _smooth_out(x, out, out_dtype)
    e = _exec(x, ex)
    with _device_guard(x):
        _lib.check(_lib.load().harpia_mean3d(_ptr(x), ic, _ptr(out), oc, _lib.i64_3(x.shape),
                                             _lib.i32_3(_triple(radius, int)), _lib.HARPIA_BORDER_REFLECT, e))
    return out


def unsharp(x, sigma, amount: float = 1.0, truncate: float = 3.0, out=None, out_dtype=None,
            ex: Exec | None = None):
    """Unsharp masking: x + amount (x - G_sigma x); output dtypes as for
    gaussian().  The Gaussian radii must be equal and at most 12."""
    ic, oc, out = _smooth_out(x, out, out_dtype)
    e = _exec(x, ex)
    with _device_guard(x):
        _lib.check(_lib.load().harpia_unsharp3d(
            _ptr(x), ic, _ptr(out), oc, _lib.i64_3(x.shape), _lib.f64_3(_triple(sigma, float)), float(truncate),
            float(amount), _lib.HARPIA_BORDER_REFLECT, e))
    return out


def local_threshold(x, method: str = "mean", radius: int = 1, sigma: float = 1.0, k: float = 0.0,
                    r_param: float = 128.0, offset: float = 0.0, truncate: float = 3.0, out=None,
                    ex: Exec | None = None):
    """Local threshold (mean, gaussian, niblack, sauvola): uint8 (x > T)."""
    _check_volume(x)
    ic = _dtype_code(x)
    if out is None:
        out = _empty_like(x, _lib.HARPIA_U8)
    else:
        _check_volume(out)
    e = _exec(x, ex)
    with _device_guard(x):
        _lib.check(_lib.load().harpia_local_threshold3d(
            _ptr(x), ic, _ptr(out), _lib.i64_3(x.shape),
            {"mean": 0, "gaussian": 1, "niblack": 2, "sauvola": 3}[method], int(radius), float(sigma),
            float(truncate), float(k), float(r_param), float(offset), _lib.HARPIA_BORDER_REFLECT, e))
    return out


def otsu(x, out=None, binarize: bool = True, ex: Exec | None = None):
    """Otsu's global threshold of a device-resident u8 / u16 volume: returns
    (uint8 (x > k) or None, k)."""
    _check_volume(x)
    ic = _dtype_code(x)
    if binarize and out is None:
        out = _empty_like(x, _lib.HARPIA_U8)
    k = _ctypes.c_int64(0)
    e = _exec(x, ex)
    with _device_guard(x):
        _lib.check(_lib.load().harpia_otsu3d(_ptr(x), ic, _ptr(out) if binarize else None, _lib.i64_3(x.shape),
                                             _ctypes.byref(k), e))
    return (out if binarize else None), int(k.value)


def hessian(x, sigma, truncate: float = 3.0, out=None, ex: Exec | None = None):
    """Hessian of the Gaussian-smoothed volume: float32 [6, nz, ny, nx] with
    components zz, zy, zx, yy, yx, xx."""
    _check_volume(x)
    ic = _dtype_code(x)
    if out is None:
        if _is_torch(x):
            out = _torch().empty((6,) + tuple(x.shape), dtype=_torch().float32, device=x.device,
                                 pin_memory=(x.device.type == "cpu" and x.is_pinned()))
        else:
            out = np.empty((6,) + tuple(x.shape), dtype=np.float32)
    e = _exec(x, ex)
    with _device_guard(x):
        _lib.check(_lib.load().harpia_hessian3d(_ptr(x), ic, _ptr(out), _lib.i64_3(x.shape),
                                                _lib.f64_3(_triple(sigma, float)), float(truncate),
                                                _lib.HARPIA_BORDER_REFLECT, e))
    return out


def edge(x, kind: str = "sobel", out=None, out_dtype=None, ex: Exec | None = None):
    """Sobel / Prewitt gradient magnitude (unnormalised weights, reflect
    boundary); output dtypes as for gaussian()."""
    ic, oc, out = _smooth_out(x, out, out_dtype)
    e = _exec(x, ex)
    with _device_guard(x):
        _lib.check(_lib.load().harpia_edge3d(_ptr(x), ic, _ptr(out), oc, _lib.i64_3(x.shape),
                                             {"sobel": 0, "prewitt": 1}[kind], _lib.HARPIA_BORDER_REFLECT, e))
    return out


def _morph_prep(x, se, radius, threshold, binary, ex, out):
    _check_volume(x)
    ic = _dtype_code(x)
    se_code = {"box": _lib.HARPIA_SE_BOX, "ball": _lib.HARPIA_SE_BALL}[se]
    thr = float("nan") if threshold is None else float(threshold)
    is_bin = binary or threshold is not None
    oc = _lib.HARPIA_U8 if is_bin else ic
    flags = _lib.HARPIA_F_BINARY if binary else 0
    if out is None:
        out = _empty_like(x, oc)
    else:
        _check_volume(out)
    return ic, se_code, _lib.i32_3(_triple(radius, int)), thr, _exec(x, ex, flags), out, oc


def erode(x, se: str = "box", radius=1, threshold=None, binary: bool = False, out=None,
          ex: Exec | None = None):
    """Erosion (min over the element).  threshold / binary: binarise the
    input (v > threshold, or v != 0) and return uint8 {0, 1}."""
    ic, sc, r, thr, e, out, _ = _morph_prep(x, se, radius, threshold, binary, ex, out)
    with _device_guard(x):
        _lib.check(_lib.load().harpia_erode3d(_ptr(x), _ptr(out), ic, _lib.i64_3(x.shape), sc, r, thr,
                                              _lib.HARPIA_BORDER_REFLECT, e))
    return out


def dilate(x, se: str = "box", radius=1, threshold=None, binary: bool = False, out=None,
           ex: Exec | None = None):
    """Dilation (max over the element); binarisation as in erode()."""
    ic, sc, r, thr, e, out, _ = _morph_prep(x, se, radius, threshold, binary, ex, out)
    with _device_guard(x):
        _lib.check(_lib.load().harpia_dilate3d(_ptr(x), _ptr(out), ic, _lib.i64_3(x.shape), sc, r, thr,
                                               _lib.HARPIA_BORDER_REFLECT, e))
    return out


def erode_dilate(x, se: str = "box", radius=1, threshold=None, binary: bool = False,
                 ex: Exec | None = None):
    """(erosion, dilation) from one read of the input."""
    ic, sc, r, thr, e, out, oc = _morph_prep(x, se, radius, threshold, binary, ex, None)
    out2 = _empty_like(x, oc)
    with _device_guard(x):
        _lib.check(_lib.load().harpia_erode_dilate3d(_ptr(x), _ptr(out), _ptr(out2), ic,
                                                     _lib.i64_3(x.shape), sc, r, thr,
                                                     _lib.HARPIA_BORDER_REFLECT, e))
    return out, out2


def morph(x, ops, se: str = "box", radius=1, threshold=None, binary: bool = False, out=None,
          ex: Exec | None = None):
    """Chain of 'erode' / 'dilate' steps with one element."""
    codes = [{"erode": _lib.HARPIA_ERODE, "dilate": _lib.HARPIA_DILATE}[o] for o in ops]
    ic, sc, r, thr, e, out, _ = _morph_prep(x, se, radius, threshold, binary, ex, out)
    arr = (ctypes_int * len(codes))(*codes)
    with _device_guard(x):
        _lib.check(_lib.load().harpia_morph3d(_ptr(x), _ptr(out), ic, _lib.i64_3(x.shape), arr,
                                              len(codes), sc, r, thr, _lib.HARPIA_BORDER_REFLECT, e))
    return out


def opening(x, se: str = "box", radius=1, threshold=None, binary: bool = False, out=None,
            ex: Exec | None = None):
    """Opening: dilation of the erosion."""
    return morph(x, ["erode", "dilate"], se, radius, threshold, binary, out, ex)


def closing(x, se: str = "box", radius=1, threshold=None, binary: bool = False, out=None,
            ex: Exec | None = None):
    """Closing: erosion of the dilation."""
    return morph(x, ["dilate", "erode"], se, radius, threshold, binary, out, ex)


def plan(shape, in_dtype="f32", out_dtype="f32", halo=(0, 0, 0), budget: int = 0,
         fraction: float = 0.0, chunk=(0, 0, 0)) -> harpia_plan:
    """Chunk plan for a streamed volume (harpia_chunk_plan)."""
    p = harpia_plan()
    e = _lib.make_exec(budget, fraction, chunk)
    _lib.check(_lib.load().harpia_chunk_plan(_lib.i64_3(shape), _code(in_dtype), _code(out_dtype),
                                            _lib.i32_3(_triple(halo, int)), e, p))
    return p


def gaussian_backward(x, grad_out, sigma, radius, grad_in=True, grad_sigma=True, ex: Exec | None = None,
                      sigma_sum: bool = False):
    """Gradients of y = gaussian(x, sigma) with the radii held fixed:
    (G^T grad_out or None, float64 tensor [3] of dL/d sigma_{z,y,x} or None).
    With sigma_sum the second is a float64 tensor [1]: the gradient of an
    isotropic sigma (the library sums the three axis terms on the device).
    Device tensors only; grad_out float32."""
    torch = _torch()
    _check_volume(grad_out)
    if grad_out.dtype != torch.float32:
        raise HarpiaError(_lib.HARPIA_ERR_DTYPE, "grad_out must be float32")
    gi = torch.empty_like(grad_out) if grad_in else None
    gs = torch.zeros(1 if sigma_sum else 3, dtype=torch.float64, device=grad_out.device) if grad_sigma else None
    xc = _dtype_code(x) if x is not None else _lib.HARPIA_F32
    e = _exec(grad_out, ex, _lib.HARPIA_F_SIGMA_SUM if sigma_sum else 0)
    with _device_guard(grad_out):
        _lib.check(_lib.load().harpia_gaussian3d_backward(
            _ptr(x) if x is not None else None, xc, _ptr(grad_out), _ptr(gi) if gi is not None else None,
            _lib.i64_3(grad_out.shape), _lib.f64_3(_triple(sigma, float)), _lib.i32_3(_triple(radius, int)),
            gs.data_ptr() if gs is not None else None, e))
    return gi, gs


def morph_backward(x, grad_out, op: str, se: str = "box", radius=1, ex: Exec | None = None):
    """Subgradient of erode/dilate(x): grad_out routed to the first extremum
    (lexicographic (dz, dy, dx) order).  Device tensors; float32 gradients."""
    torch = _torch()
    _check_volume(x)
    _check_volume(grad_out)
    gi = torch.empty_like(grad_out)
    code = {"erode": _lib.HARPIA_ERODE, "dilate": _lib.HARPIA_DILATE}[op]
    sc = {"box": _lib.HARPIA_SE_BOX, "ball": _lib.HARPIA_SE_BALL}[se]
    e = _exec(grad_out, ex)
    with _device_guard(grad_out):
        _lib.check(_lib.load().harpia_morph3d_backward(
            _ptr(x), _dtype_code(x), _ptr(grad_out), _ptr(gi), _lib.i64_3(x.shape), code, sc,
            _lib.i32_3(_triple(radius, int)), e))
    return gi


def _sigma_values(sigma):
    torch = _torch()
    if isinstance(sigma, torch.Tensor):
        vals = sigma.detach().double().cpu().reshape(-1).tolist()
        return (vals[0],) * 3 if len(vals) == 1 else tuple(vals)
    return _triple(sigma, float)


def _sigma_grad(sigma, gs):
    """dL/d sigma in the shape of `sigma` (gs from gaussian_backward, with
    sigma_sum for a one-element sigma)."""
    if gs is None:
        return None
    return gs.to(device=sigma.device, dtype=sigma.dtype).reshape(sigma.shape)


def _autograd_base():
    return _torch().autograd.Function


class _LazyFunction(type):
    """Builds the torch.autograd.Function subclass on first use, so that the
    package imports without torch's autograd machinery being touched."""

    def __getattr__(cls, name):
        return getattr(cls._impl(), name)


class GaussianFn(metaclass=_LazyFunction):
    """y = G_sigma x as an autograd Function: GaussianFn.apply(x, sigma,
    truncate).  sigma: float, triple, or a (learnable) tensor with 1 or 3
    elements.  The radius is resolved from sigma in forward and held fixed
    in backward; only x is saved."""
    _cls = None

    @classmethod
    def _impl(cls):
        if cls._cls is None:
            torch = _torch()

            class _Fn(torch.autograd.Function):
                @staticmethod
                def forward(ctx, x, sigma, truncate=3.0):
                    s = _sigma_values(sigma)
                    r = tuple(gauss_radius(t, truncate) for t in s)
                    ctx.save_for_backward(x, sigma if isinstance(sigma, torch.Tensor) else None)
                    ctx.s, ctx.r = s, r
                    return gaussian(x.detach().contiguous(), s, truncate)

                @staticmethod
                def backward(ctx, gy):
                    x, sig = ctx.saved_tensors
                    need_s = sig is not None and ctx.needs_input_grad[1]
                    gx, gs = gaussian_backward(x.contiguous(), gy.contiguous().float(), ctx.s, ctx.r,
                                               grad_in=ctx.needs_input_grad[0], grad_sigma=need_s,
                                               sigma_sum=need_s and sig.numel() == 1)
                    return (gx.to(x.dtype) if gx is not None else None,
                            _sigma_grad(sig, gs) if need_s else None, None)

            cls._cls = _Fn
        return cls._cls


class MorphFn(metaclass=_LazyFunction):
    """Erosion / dilation as an autograd Function: MorphFn.apply(x, op, se,
    radius) with op 'erode' or 'dilate'; the gradient routes to the first
    extremum.  Saves x only."""
    _cls = None

    @classmethod
    def _impl(cls):
        if cls._cls is None:
            torch = _torch()

            class _Fn(torch.autograd.Function):
                @staticmethod
                def forward(ctx, x, op, se="box", radius=1):
                    ctx.save_for_backward(x)
                    ctx.args = (op, se, radius)
                    f = erode if op == "erode" else dilate
                    return f(x.detach().contiguous(), se, radius)

                @staticmethod
                def backward(ctx, gy):
                    (x,) = ctx.saved_tensors
                    op, se, radius = ctx.args
                    return morph_backward(x.contiguous(), gy.contiguous().float(), op, se, radius), None, None, None

            cls._cls = _Fn
        return cls._cls


class GaussDilateFn(metaclass=_LazyFunction):
    """d = dilate_se(G_sigma x) in one autograd node that stores only x and
    sigma: backward recomputes y = G_sigma x, routes the upstream gradient
    through the dilation's first maxima, then applies the Gaussian's adjoint
    and sigma-gradient.  GaussDilateFn.apply(x, sigma, se, radius, truncate)."""
    _cls = None

    @classmethod
    def _impl(cls):
        if cls._cls is None:
            torch = _torch()

            class _Fn(torch.autograd.Function):
                @staticmethod
                def forward(ctx, x, sigma, se="box", radius=2, truncate=3.0):
                    s = _sigma_values(sigma)
                    r = tuple(gauss_radius(t, truncate) for t in s)
                    ctx.save_for_backward(x, sigma if isinstance(sigma, torch.Tensor) else None)
                    ctx.s, ctx.r, ctx.m, ctx.t = s, r, (se, radius), truncate
                    y = gaussian(x.detach().contiguous(), s, truncate)
                    return dilate(y, se, radius)

                @staticmethod
                def backward(ctx, gd):
                    x, sig = ctx.saved_tensors
                    se, radius = ctx.m
                    y = gaussian(x.contiguous(), ctx.s, ctx.t)  # recomputed, not stored
                    gy = morph_backward(y, gd.contiguous().float(), "dilate", se, radius)
                    del y
                    need_s = sig is not None and ctx.needs_input_grad[1]
                    gx, gs = gaussian_backward(x.contiguous(), gy, ctx.s, ctx.r,
                                               grad_in=ctx.needs_input_grad[0], grad_sigma=need_s,
                                               sigma_sum=need_s and sig.numel() == 1)
                    return (gx.to(x.dtype) if gx is not None else None,
                            _sigma_grad(sig, gs) if need_s else None, None, None, None)

            cls._cls = _Fn
        return cls._cls


def _stream():
    return _torch().cuda.current_stream().cuda_stream


def gaussian_batched(xs, sigma, truncate: float = 3.0, outs=None):
    """Gaussian of every crop in one persistent launch per 64 crops (float32
    device tensors of any shapes; equal radii 1..12)."""
    torch = _torch()
    outs = [torch.empty_like(x) for x in xs] if outs is None else outs
    arr = _lib.crops([(x, o, None) for x, o in zip(xs, outs)])
    _lib.check(_lib.load().harpia_gaussian3d_batched(arr, len(xs), _lib.HARPIA_F32, _lib.HARPIA_F32,
                                                     _lib.f64_3(_triple(sigma, float)), float(truncate),
                                                     _lib.make_exec(stream=_stream())))
    return outs


def morph_batched(xs, op: str, se: str = "box", radius=1, outs=None, outs2=None):
    """Erosion / dilation of every crop (float32); with outs2 given, outs get
    the erosion and outs2 the dilation from one launch."""
    torch = _torch()
    outs = [torch.empty_like(x) for x in xs] if outs is None else outs
    aux = outs2 if outs2 is not None else [None] * len(xs)
    arr = _lib.crops([(x, o, a) for x, o, a in zip(xs, outs, aux)])
    _lib.check(_lib.load().harpia_morph3d_batched(
        arr, len(xs), _lib.HARPIA_F32, {"erode": _lib.HARPIA_ERODE, "dilate": _lib.HARPIA_DILATE}[op],
        {"box": _lib.HARPIA_SE_BOX, "ball": _lib.HARPIA_SE_BALL}[se], _lib.i32_3(_triple(radius, int)),
        _lib.make_exec(stream=_stream())))
    return outs


class GaussDilateBatch:
    """Forward and backward of d_i = dilate_se(G_sigma x_i) over a fixed list
    of float32 crops (the differentiable batched workload), with every buffer
    allocated up front so that a step allocates nothing and can be captured
    in a CUDA/HIP graph:

        fwd:  y = G x (batched), d = dilate(y) with the codes of the maxima
              kept in the workspace (one batched pass)
        bwd:  g_y = g_d routed through the kept codes (batched gather),
              g_x = G g_y (batched), d L / d sigma = sum_a <g_y, G'_a x>
              (batched dot, FP64 reduction, the three axis terms summed
              on the device) -- kept on the device.
    Six launches per step.  sigma is a Python float (isotropic); its radius
    is resolved once."""

    def __init__(self, xs, sigma: float, se: str = "box", radius=2, truncate: float = 3.0):
        torch = _torch()
        self.xs = xs
        self.sigma = float(sigma)
        self.truncate = float(truncate)
        self.r = gauss_radius(self.sigma, truncate)
        self.se, self.mr = se, radius
        self.ys = [torch.empty_like(x) for x in xs]
        self.ds = [torch.empty_like(x) for x in xs]
        self.gys = [torch.empty_like(x) for x in xs]
        self.gxs = [torch.empty_like(x) for x in xs]
        self.gsigma = torch.zeros(1, dtype=torch.float64, device=xs[0].device)
        self._c_fwd_g = _lib.crops([(x, y, None) for x, y in zip(xs, self.ys)])
        self._c_fwd_d = _lib.crops([(y, d, None) for y, d in zip(self.ys, self.ds)])
        nbytes = _lib.load().harpia_batch_workspace_bytes(self._c_fwd_g, len(xs))
        self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=xs[0].device)
        self.gds = None

    def forward(self):
        lib, n, st = _lib.load(), len(self.xs), _lib.make_exec(stream=_stream())
        s3 = _lib.f64_3((self.sigma,) * 3)
        _lib.check(lib.harpia_gaussian3d_batched(self._c_fwd_g, n, _lib.HARPIA_F32, _lib.HARPIA_F32, s3,
                                                 self.truncate, st))
        _lib.check(lib.harpia_morph3d_forward_batched(self._c_fwd_d, n, _lib.HARPIA_DILATE,
                                                      {"box": 0, "ball": 1}[self.se],
                                                      _lib.i32_3(_triple(self.mr, int)), self.workspace.data_ptr(),
                                                      self.workspace.numel(), st))
        return self.ds

    def backward(self, gds):
        """gds: upstream gradients (float32 tensors like the crops).  Returns
        (grad_x list, dL/dsigma of the isotropic sigma as a float64 device
        tensor [1])."""
        lib, n = _lib.load(), len(self.xs)
        st_sum = _lib.make_exec(stream=_stream(), flags=_lib.HARPIA_F_SIGMA_SUM)
        st_reuse = _lib.make_exec(stream=_stream(), flags=_lib.HARPIA_F_REUSE_CODES)
        if self.gds is not gds:
            self.gds = gds
            self._c_bwd_m = _lib.crops([(None, gy, g) for gy, g in zip(self.gys, gds)])
            self._c_bwd_g = _lib.crops([(x, gx, gy) for x, gx, gy in zip(self.xs, self.gxs, self.gys)])
        s3 = _lib.f64_3((self.sigma,) * 3)
        r3 = _lib.i32_3((self.r,) * 3)
        ws, wsb = self.workspace.data_ptr(), self.workspace.numel()
        # route through the codes the forward kept (no recomputation of y)
        _lib.check(lib.harpia_morph3d_backward_batched(self._c_bwd_m, n, _lib.HARPIA_DILATE,
                                                       {"box": 0, "ball": 1}[self.se],
                                                       _lib.i32_3(_triple(self.mr, int)), ws, wsb, st_reuse))
        _lib.check(lib.harpia_gaussian3d_backward_batched(self._c_bwd_g, n, s3, r3, self.gsigma.data_ptr(), ws,
                                                          wsb, st_sum))
        return self.gxs, self.gsigma

    def autotune(self, reps: int = 3):
        """Pick the tiles of every batched kernel of this pipeline on these
        crops (the library's autotuner; y and g_y buffers are used as
        scratch).  Returns the tuner's report, one dict per kernel."""
        lib, n, st = _lib.load(), len(self.xs), _lib.make_exec(stream=_stream())
        c = _lib.crops([(x, y, gy) for x, y, gy in zip(self.xs, self.ys, self.gys)])
        rep = _lib.harpia_tune_report()
        _lib.check(lib.harpia_autotune_gauss_dilate_batched(
            c, n, _lib.f64_3((self.sigma,) * 3), _lib.i32_3((self.r,) * 3), {"box": 0, "ball": 1}[self.se],
            _lib.i32_3(_triple(self.mr, int)), self.workspace.data_ptr(), self.workspace.numel(), int(reps), st,
            _ctypes.byref(rep)))
        return rep.entries()


def autotune_gaussian(x, sigma, out=None, truncate: float = 3.0, reps: int = 3):
    """Autotune the fused Gaussian on this device-resident volume (out is
    overwritten); later calls with the same shape, dtype and radius use the
    chosen z split.  Returns the tuner's report."""
    torch = _torch()
    out = torch.empty_like(x) if out is None else out
    rep = _lib.harpia_tune_report()
    _lib.check(_lib.load().harpia_autotune_gaussian3d(
        x.data_ptr(), _dtype_code(x), out.data_ptr(), _dtype_code(out), _lib.i64_3(x.shape),
        _lib.f64_3(_triple(sigma, float)), float(truncate), int(reps), _lib.make_exec(stream=_stream()),
        _ctypes.byref(rep)))
    return rep.entries()


def autotune_erode_dilate(x, se: str = "ball", radius=1, ero=None, dil=None, reps: int = 3,
                          threshold=None, binary: bool = False):
    """Autotune the erosion+dilation kernel on this volume (grayscale, or
    binary with a threshold or binary=True; outputs then uint8)."""
    torch = _torch()
    bin_out = binary or threshold is not None
    ero = (torch.empty_like(x, dtype=torch.uint8) if bin_out else torch.empty_like(x)) if ero is None else ero
    dil = (torch.empty_like(x, dtype=torch.uint8) if bin_out else torch.empty_like(x)) if dil is None else dil
    rep = _lib.harpia_tune_report()
    _lib.check(_lib.load().harpia_autotune_erode_dilate3d(
        x.data_ptr(), ero.data_ptr(), dil.data_ptr(), _dtype_code(x), _lib.i64_3(x.shape),
        {"box": 0, "ball": 1}[se], _lib.i32_3(_triple(radius, int)),
        float("nan") if threshold is None else float(threshold), int(reps),
        _lib.make_exec(stream=_stream(), flags=_lib.HARPIA_F_BINARY if binary else 0), _ctypes.byref(rep)))
    return rep.entries()


def tune_clear():
    _lib.check(_lib.load().harpia_tune_clear())


def tune_entries() -> int:
    return int(_lib.load().harpia_tune_entries())


def tune_save(path: str):
    _lib.check(_lib.load().harpia_tune_save(str(path).encode()))


def tune_load(path: str):
    _lib.check(_lib.load().harpia_tune_load(str(path).encode()))


import ctypes as _ctypes  # noqa: E402

ctypes_int = _ctypes.c_int
