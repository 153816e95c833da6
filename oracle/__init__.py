"""FP64 CPU oracle for the Harpia volumetric filters.

TEST INFRASTRUCTURE ONLY: the test-suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` are the only callers.  The product path
(the ``paper_2511_11890_amd`` package and its HIP library) never imports this
module, and this module never imports the product path.

The arithmetic lives in ``oracle.c`` (plain C, FP64, OpenMP over z); this file
only marshals numpy arrays and composes the C primitives into the operations
the paper names (Section III-C: Gaussian smoothing, erosion, dilation,
opening, closing; thresholding from the label-editing module).  Every
definition is the plain textbook one; the readings adopted where the paper is
silent are listed in the header of ``oracle.c``.

Parity pins: ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc into liboracle.so (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
               "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    i64p = ctypes.POINTER(ctypes.c_int64)
    ip = ctypes.POINTER(ctypes.c_int)
    lib.oracle_reflect.argtypes = [ctypes.c_int64, ctypes.c_int64]
    lib.oracle_reflect.restype = ctypes.c_int64
    lib.oracle_gauss_radius.argtypes = [ctypes.c_double, ctypes.c_double]
    lib.oracle_gauss_radius.restype = ctypes.c_int
    lib.oracle_gauss_taps.argtypes = [ctypes.c_double, ctypes.c_int, dp]
    lib.oracle_gauss_taps.restype = ctypes.c_int
    lib.oracle_gauss_dtaps.argtypes = [ctypes.c_double, ctypes.c_int, dp]
    lib.oracle_gauss_dtaps.restype = ctypes.c_int
    conv_args = [dp, dp, i64p, dp, ctypes.c_int, dp, ctypes.c_int, dp, ctypes.c_int]
    lib.oracle_conv3d_direct.argtypes = conv_args
    lib.oracle_conv3d_direct.restype = None
    lib.oracle_conv3d_separable.argtypes = conv_args
    lib.oracle_conv3d_separable.restype = ctypes.c_int
    lib.oracle_conv3d_transpose.argtypes = conv_args
    lib.oracle_conv3d_transpose.restype = ctypes.c_int
    lib.oracle_conv1d.argtypes = [dp, dp, i64p, ctypes.c_int, dp, ctypes.c_int]
    lib.oracle_conv1d.restype = None
    lib.oracle_conv1d_transpose.argtypes = [dp, dp, i64p, ctypes.c_int, dp, ctypes.c_int]
    lib.oracle_conv1d_transpose.restype = None
    lib.oracle_morph3d.argtypes = [dp, dp, i64p, i64p, ctypes.c_int, ctypes.c_int, ip]
    lib.oracle_morph3d.restype = ctypes.c_int
    lib.oracle_route.argtypes = [dp, i64p, dp, ctypes.c_int64]
    lib.oracle_route.restype = None
    lib.oracle_threshold.argtypes = [dp, dp, ctypes.c_int64, ctypes.c_double]
    lib.oracle_threshold.restype = None
    lib.oracle_num_threads.argtypes = []
    lib.oracle_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _f64(a) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if a.ndim != 3:
        raise ValueError("oracle volumes are 3D [nz, ny, nx]")
    return a


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i64p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _shape(a: np.ndarray) -> np.ndarray:
    return np.array(a.shape, dtype=np.int64)


def _triple(v, cast):
    if np.ndim(v) == 0:
        return (cast(v),) * 3
    v = tuple(cast(t) for t in v)
    if len(v) != 3:
        raise ValueError("expected a scalar or a (z, y, x) triple")
    return v


# ---------------------------------------------------------------- scalars

def reflect(i: int, n: int) -> int:
    """Half-sample symmetric reflection of index i into [0, n)."""
    return int(_load().oracle_reflect(int(i), int(n)))


def gauss_radius(sigma: float, truncate: float = 3.0) -> int:
    """r = int(truncate * sigma + 0.5)."""
    return int(_load().oracle_gauss_radius(float(sigma), float(truncate)))


def gauss_taps(sigma: float, r: int) -> np.ndarray:
    """Normalised sampled Gaussian taps w[k + r], k = -r..r (FP64)."""
    w = np.empty(2 * r + 1, dtype=np.float64)
    if _load().oracle_gauss_taps(float(sigma), int(r), _dp(w)) != 0:
        raise ValueError("sigma must be > 0 and r >= 0")
    return w


def gauss_dtaps(sigma: float, r: int) -> np.ndarray:
    """d w[k + r] / d sigma with r held fixed (FP64)."""
    w = np.empty(2 * r + 1, dtype=np.float64)
    if _load().oracle_gauss_dtaps(float(sigma), int(r), _dp(w)) != 0:
        raise ValueError("sigma must be > 0 and r >= 0")
    return w


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_threads(n: int) -> None:
    """Worker threads of later oracle calls from this thread (OpenMP's
    omp_set_num_threads of the runtime the oracle is linked against); used
    to time the oracle on one core and on all cores."""
    _load()
    ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))


# ---------------------------------------------------------------- Gaussian

def _radii(sigma, truncate, radius):
    s = _triple(sigma, float)
    if radius is None:
        r = tuple(gauss_radius(si, truncate) for si in s)
    else:
        r = _triple(radius, int)
    return s, r


def _taps3(s, r, deriv_axis=None):
    return [gauss_dtaps(s[a], r[a]) if a == deriv_axis else gauss_taps(s[a], r[a])
            for a in range(3)]


def conv3d(v, wz, wy, wx, method: str = "separable") -> np.ndarray:
    """Convolve with the outer product wz x wy x wx (odd lengths, centred)."""
    v = _f64(v)
    out = np.empty_like(v)
    taps = [np.ascontiguousarray(w, dtype=np.float64) for w in (wz, wy, wx)]
    rs = [(len(w) - 1) // 2 for w in taps]
    lib = _load()
    args = (_dp(v), _dp(out), _i64p(_shape(v)),
            _dp(taps[0]), rs[0], _dp(taps[1]), rs[1], _dp(taps[2]), rs[2])
    if method == "direct":
        lib.oracle_conv3d_direct(*args)
    elif method == "separable":
        if lib.oracle_conv3d_separable(*args) != 0:
            raise MemoryError("oracle allocation failed")
    elif method == "transpose":
        if lib.oracle_conv3d_transpose(*args) != 0:
            raise MemoryError("oracle allocation failed")
    else:
        raise ValueError(method)
    return out


def gaussian3d(v, sigma, truncate: float = 3.0, radius=None,
               method: str = "direct") -> np.ndarray:
    """Gaussian smoothing with half-sample reflect boundary.

    ``method='direct'`` is the triple loop over taps (the definition);
    ``'separable'`` runs three 1D passes (pinned equal to 'direct').
    ``radius`` overrides the truncation radius (used to hold r fixed)."""
    s, r = _radii(sigma, truncate, radius)
    wz, wy, wx = _taps3(s, r)
    return conv3d(v, wz, wy, wx, method=method)


def gaussian3d_transpose(g, sigma, truncate: float = 3.0, radius=None) -> np.ndarray:
    """G^T g by literal scatter of every forward product (adjoint)."""
    s, r = _radii(sigma, truncate, radius)
    wz, wy, wx = _taps3(s, r)
    return conv3d(g, wz, wy, wx, method="transpose")


def gaussian3d_dsigma_axis(v, sigma, axis: int, truncate: float = 3.0,
                           radius=None) -> np.ndarray:
    """d/d sigma_axis of (G_sigma v), radii held fixed: the separable
    convolution with dw on `axis` and w on the other two axes."""
    s, r = _radii(sigma, truncate, radius)
    wz, wy, wx = _taps3(s, r, deriv_axis=axis)
    return conv3d(v, wz, wy, wx, method="separable")


def gaussian3d_dsigma(v, sigma: float, truncate: float = 3.0, radius=None) -> np.ndarray:
    """d/d sigma of (G_sigma v) for an isotropic sigma shared by all axes:
    the sum of the three per-axis derivatives (chain rule)."""
    return sum(gaussian3d_dsigma_axis(v, sigma, a, truncate, radius) for a in range(3))


# ---------------------------------------------------------------- morphology

_SE = {"box": 0, "ball": 1}


def morph3d(v, op: str, se: str = "box", radius=1, return_arg: bool = False):
    """Erosion (op='erode', min) or dilation (op='dilate', max) by brute
    force over the structuring element, out-of-volume offsets skipped.
    With return_arg, also the flat index of the first extremum in
    lexicographic (dz, dy, dx) order."""
    v = _f64(v)
    out = np.empty_like(v)
    arg = np.empty(v.shape, dtype=np.int64) if return_arg else None
    r = np.array(_triple(radius, int), dtype=np.int32)
    code = {"erode": 0, "dilate": 1}[op]
    rc = _load().oracle_morph3d(
        _dp(v), _dp(out), _i64p(arg) if arg is not None else None,
        _i64p(_shape(v)), code, _SE[se],
        r.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    if rc != 0:
        raise ValueError("invalid morphology arguments")
    return (out, arg) if return_arg else out


def erode3d(v, se="box", radius=1):
    return morph3d(v, "erode", se, radius)


def dilate3d(v, se="box", radius=1):
    return morph3d(v, "dilate", se, radius)


def threshold(v, t: float) -> np.ndarray:
    """b = 1.0 where v > t (strict), else 0.0."""
    v = _f64(v)
    b = np.empty_like(v)
    _load().oracle_threshold(_dp(v), _dp(b), v.size, float(t))
    return b


def mean3d(v, radius=1, method: str = "direct") -> np.ndarray:
    """Mean (box) filter of the filtering suite (Section III-C): the average
    over the (2r+1)-box per axis, reflect boundary -- the convolution with
    uniform taps 1/(2r+1) on each axis."""
    r = _triple(radius, int)
    taps = [np.full(2 * ri + 1, 1.0 / (2 * ri + 1)) for ri in r]
    return conv3d(v, taps[0], taps[1], taps[2], method=method)


def unsharp3d(v, sigma, amount: float, truncate: float = 3.0) -> np.ndarray:
    """Unsharp masking (Section III-C): the input plus `amount` times its
    difference from the Gaussian-smoothed input, v + a (v - G_sigma v)."""
    v = _f64(v)
    return v + float(amount) * (v - gaussian3d(v, sigma, truncate, method="direct"))


def edge3d_axes(v, kind: str = "sobel"):
    """The three per-axis responses of the Sobel / Prewitt operator
    (Section III-C, edge enhancement): along axis a the central difference
    [-1, 0, 1] (v[i+1] - v[i-1]), along the other two axes the smoothing
    [1, 2, 1] (Sobel) or [1, 1, 1] (Prewitt); reflect boundary."""
    sm = np.array([1.0, 2.0, 1.0]) if kind == "sobel" else np.array([1.0, 1.0, 1.0])
    d = np.array([-1.0, 0.0, 1.0])
    return [conv3d(v, *[d if b == a else sm for b in range(3)], method="direct") for a in range(3)]


def edge3d(v, kind: str = "sobel") -> np.ndarray:
    """Gradient magnitude sqrt(Gz^2 + Gy^2 + Gx^2) of the Sobel / Prewitt
    operator (unnormalised weights)."""
    gz, gy, gx = edge3d_axes(v, kind)
    return np.sqrt(gz * gz + gy * gy + gx * gx)


def gauss_deriv_taps(sigma: float, r: int, order: int) -> np.ndarray:
    """Correlation taps c[k + r] of the order-th derivative of the Gaussian
    smoothing along one axis: with w the normalised taps, c = w (order 0),
    (k / s^2) w (order 1: d/dx of the smoothed signal, v[i + k] weighted by
    c[k]), ((k^2 - s^2) / s^4) w (order 2)."""
    w = gauss_taps(sigma, r)
    k = np.arange(-r, r + 1, dtype=np.float64)
    s2 = float(sigma) ** 2
    if order == 0:
        return w
    if order == 1:
        return k / s2 * w
    if order == 2:
        return (k * k - s2) / (s2 * s2) * w
    raise ValueError("order must be 0, 1 or 2")


HESSIAN_PAIRS = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))


def hessian3d(v, sigma, truncate: float = 3.0) -> np.ndarray:
    """Hessian of the Gaussian-smoothed volume (Section III-C texture
    features): components zz, zy, zx, yy, yx, xx, each the separable
    correlation with derivative taps of the orders the pair asks for;
    reflect boundary.  Returns an array [6, nz, ny, nx]."""
    s = _triple(sigma, float)
    r = tuple(gauss_radius(si, truncate) for si in s)
    out = []
    for a, b in HESSIAN_PAIRS:
        orders = [0, 0, 0]
        orders[a] += 1
        orders[b] += 1
        taps = [gauss_deriv_taps(s[i], r[i], orders[i]) for i in range(3)]
        out.append(conv3d(v, *taps, method="direct"))
    return np.stack(out)


THRESHOLD_METHODS = ("mean", "gaussian", "niblack", "sauvola")


def local_threshold3d(v, method: str, radius=1, sigma: float = 1.0, k: float = 0.0, r_param: float = 128.0,
                      offset: float = 0.0, return_t: bool = False):
    """Local thresholds of the label-editing module (Section III-C), each
    voxel against a threshold T from its neighbourhood (reflect boundary):
      mean:     T = m - offset, m the (2r+1)-box mean;
      gaussian: T = G_sigma v - offset;
      niblack:  T = m + k s, s the box standard deviation
                sqrt(mean(v^2) - m^2) (population form);
      sauvola:  T = m (1 + k (s / r_param - 1)).
    Returns uint8 (v > T), and T with return_t."""
    v = _f64(v)
    if method == "gaussian":
        t = gaussian3d(v, sigma, method="direct") - offset
    else:
        m = mean3d(v, radius, method="direct")
        if method == "mean":
            t = m - offset
        else:
            q = mean3d(v * v, radius, method="direct")
            sd = np.sqrt(np.maximum(q - m * m, 0.0))
            if method == "niblack":
                t = m + k * sd
            elif method == "sauvola":
                t = m * (1.0 + k * (sd / r_param - 1.0))
            else:
                raise ValueError("unknown method")
    out = (v > t).astype(np.uint8)
    return (out, t) if return_t else out


def otsu_threshold(v, nbins: int) -> int:
    """Otsu's global threshold (Section III-C threshold algorithms) over the
    integer histogram of v (one bin per value 0 .. nbins - 1): the split k
    (class 0: values <= k) maximising the between-class variance
    w0 w1 (m0 - m1)^2, w the class counts and m the class means, evaluated
    in FP64 in this order from exact integer sums; the first maximum wins.
    Returns -1 when every voxel holds one value."""
    v = np.asarray(v).ravel().astype(np.int64)
    counts = np.bincount(v, minlength=nbins)[:nbins].astype(np.int64)
    n = int(counts.sum())
    total = int(np.dot(np.arange(nbins, dtype=np.int64), counts))
    best_k, best = -1, -1.0
    c0 = s0 = 0
    for k in range(nbins - 1):
        c0 += int(counts[k])
        s0 += k * int(counts[k])
        c1 = n - c0
        if c0 == 0 or c1 == 0:
            continue
        d = float(s0) / float(c0) - float(total - s0) / float(c1)
        sb = (float(c0) * float(c1)) * (d * d)
        if sb > best:
            best, best_k = sb, k
    return best_k


def otsu3d(v, nbins: int) -> np.ndarray:
    """uint8 (v > k) with k = otsu_threshold(v)."""
    k = otsu_threshold(v, nbins)
    return (np.asarray(v).astype(np.int64) > k).astype(np.uint8)


def opening3d(v, se="box", radius=1):
    """Opening = dilation of the erosion, each over the full volume."""
    return dilate3d(erode3d(v, se, radius), se, radius)


def closing3d(v, se="box", radius=1):
    """Closing = erosion of the dilation, each over the full volume."""
    return erode3d(dilate3d(v, se, radius), se, radius)


def morph3d_backward(v, g, op: str, se="box", radius=1) -> np.ndarray:
    """Subgradient of erosion/dilation: route g[p] to the first extremum."""
    _, arg = morph3d(v, op, se, radius, return_arg=True)
    g = _f64(g)
    gin = np.empty_like(g)
    _load().oracle_route(_dp(g), _i64p(arg), _dp(gin), g.size)
    return gin


# ---------------------------------------------------------------- composite

def gauss_dilate_loss_grad(x, c, sigma: float, se="box", radius=2,
                           truncate: float = 3.0, gauss_radius_fixed=None):
    """L = sum_p c_p * dilate(G_sigma x)(p) with isotropic sigma.

    Returns (L, dL/dx, dL/dsigma, y) where y = G_sigma x.  The Gaussian
    radius is resolved once from sigma (or given) and held fixed."""
    x = _f64(x)
    c = _f64(c)
    r = gauss_radius(sigma, truncate) if gauss_radius_fixed is None else int(gauss_radius_fixed)
    y = gaussian3d(x, sigma, radius=r, method="separable")
    d, arg = morph3d(y, "dilate", se, radius, return_arg=True)
    loss = float(np.sum(c * d))
    gy = np.empty_like(c)
    _load().oracle_route(_dp(c), _i64p(arg), _dp(gy), c.size)
    gx = gaussian3d_transpose(gy, sigma, radius=r)
    gs = float(np.sum(gy * gaussian3d_dsigma(x, sigma, radius=r)))
    return loss, gx, gs, y
