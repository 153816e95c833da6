"""ctypes binding of libharpia (include/harpia.h): names, structs and
signatures mirror the header one to one; this module only marshals
arguments.  Every filter runs in the HIP library; there is no Python or CPU
fallback, and loading fails loudly if the library has not been built."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libharpia.so")

# harpia_status
HARPIA_OK = 0
HARPIA_ERR_ARG = -1
HARPIA_ERR_DTYPE = -2
HARPIA_ERR_BUDGET = -3
HARPIA_ERR_OOM = -4
HARPIA_ERR_HIP = -5
HARPIA_ERR_ALIAS = -6
HARPIA_ERR_UNSUPPORTED = -7
STATUS_NAMES = {
    0: "HARPIA_OK", -1: "HARPIA_ERR_ARG", -2: "HARPIA_ERR_DTYPE", -3: "HARPIA_ERR_BUDGET",
    -4: "HARPIA_ERR_OOM", -5: "HARPIA_ERR_HIP", -6: "HARPIA_ERR_ALIAS", -7: "HARPIA_ERR_UNSUPPORTED",
}

# harpia_dtype
HARPIA_U8, HARPIA_U16, HARPIA_F32, HARPIA_F16, HARPIA_BF16 = 0, 1, 2, 3, 4
# harpia_se
HARPIA_SE_BOX, HARPIA_SE_BALL = 0, 1
# harpia_border
HARPIA_BORDER_REFLECT = 0
# harpia_morph_op
HARPIA_ERODE, HARPIA_DILATE = 0, 1
# flags
HARPIA_F_BINARY = 0x1
HARPIA_F_FORCE_CHUNKED = 0x2
HARPIA_F_SIGMA_SUM = 0x4
HARPIA_F_REUSE_CODES = 0x8


class harpia_stats(ctypes.Structure):
    _fields_ = [("n_chunks", ctypes.c_int64), ("bytes_h2d", ctypes.c_int64),
                ("bytes_d2h", ctypes.c_int64), ("peak_device_bytes", ctypes.c_int64),
                ("budget_bytes", ctypes.c_int64), ("wall_ms", ctypes.c_double),
                ("kernel_ms", ctypes.c_double)]


class harpia_exec(ctypes.Structure):
    _fields_ = [("device_budget_bytes", ctypes.c_size_t), ("budget_fraction", ctypes.c_double),
                ("chunk", ctypes.c_int64 * 3), ("stream", ctypes.c_void_p),
                ("flags", ctypes.c_uint32), ("stats", ctypes.POINTER(harpia_stats))]


class harpia_plan(ctypes.Structure):
    _fields_ = [("shape", ctypes.c_int64 * 3), ("core", ctypes.c_int64 * 3),
                ("grid", ctypes.c_int64 * 3), ("halo", ctypes.c_int32 * 3),
                ("n_buffers", ctypes.c_int32), ("n_chunks", ctypes.c_int64),
                ("device_bytes", ctypes.c_size_t), ("budget_bytes", ctypes.c_size_t)]


class harpia_crop(ctypes.Structure):
    _fields_ = [("in_", ctypes.c_void_p), ("out", ctypes.c_void_p), ("aux", ctypes.c_void_p),
                ("shape", ctypes.c_int64 * 3)]


class harpia_tune_entry(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_char * 24), ("tile", ctypes.c_int32 * 3), ("candidates", ctypes.c_int32),
                ("ms_heuristic", ctypes.c_float), ("ms_best", ctypes.c_float)]


class harpia_tune_report(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("e", harpia_tune_entry * 8)]

    def entries(self):
        return [{"kernel": self.e[i].kernel.decode(), "tile": tuple(self.e[i].tile),
                 "candidates": self.e[i].candidates, "ms_heuristic": round(self.e[i].ms_heuristic, 4),
                 "ms_best": round(self.e[i].ms_best, 4)} for i in range(self.n)]


class HarpiaError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, str(status)), message))
        self.status = status
        self.message = message


_I64_3 = ctypes.c_int64 * 3
_I32_3 = ctypes.c_int32 * 3
_F64_3 = ctypes.c_double * 3
_vp = ctypes.c_void_p
_ex = ctypes.POINTER(harpia_exec)

# name -> (restype, argtypes); the order follows include/harpia.h
SIGNATURES = {
    "harpia_last_error": (ctypes.c_char_p, []),
    "harpia_version": (ctypes.c_char_p, []),
    "harpia_gauss_radius": (ctypes.c_int32, [ctypes.c_double, ctypes.c_double]),
    "harpia_chunk_plan": (ctypes.c_int, [_I64_3, ctypes.c_int, ctypes.c_int, _I32_3, _ex,
                                         ctypes.POINTER(harpia_plan)]),
    "harpia_gaussian3d": (ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.c_int, _I64_3, _F64_3,
                                         ctypes.c_double, ctypes.c_int, _ex]),
    "harpia_mean3d": (ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.c_int, _I64_3, _I32_3, ctypes.c_int, _ex]),
    "harpia_otsu3d": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _I64_3, ctypes.POINTER(ctypes.c_int64), _ex]),
    "harpia_local_threshold3d": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _I64_3, ctypes.c_int, ctypes.c_int32,
                                                ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                                ctypes.c_double, ctypes.c_int, _ex]),
    "harpia_hessian3d": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _I64_3, _F64_3, ctypes.c_double, ctypes.c_int,
                                        _ex]),
    "harpia_edge3d": (ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.c_int, _I64_3, ctypes.c_int, ctypes.c_int, _ex]),
    "harpia_unsharp3d": (ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.c_int, _I64_3, _F64_3, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_int, _ex]),
    "harpia_erode3d": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _I64_3, ctypes.c_int, _I32_3,
                                      ctypes.c_double, ctypes.c_int, _ex]),
    "harpia_dilate3d": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _I64_3, ctypes.c_int, _I32_3,
                                       ctypes.c_double, ctypes.c_int, _ex]),
    "harpia_erode_dilate3d": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _I64_3, ctypes.c_int,
                                             _I32_3, ctypes.c_double, ctypes.c_int, _ex]),
    "harpia_morph3d": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _I64_3, ctypes.POINTER(ctypes.c_int),
                                      ctypes.c_int32, ctypes.c_int, _I32_3, ctypes.c_double,
                                      ctypes.c_int, _ex]),
    "harpia_gaussian3d_backward": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _I64_3, _F64_3, _I32_3,
                                                  _vp, _ex]),
    "harpia_gaussian3d_backward_noalloc": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _I64_3, _F64_3, _I32_3,
                                                          _vp, _ex]),
    "harpia_morph3d_backward": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _I64_3, ctypes.c_int,
                                               ctypes.c_int, _I32_3, _ex]),
    "harpia_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(harpia_crop), ctypes.c_int32]),
    "harpia_gaussian3d_batched": (ctypes.c_int, [ctypes.POINTER(harpia_crop), ctypes.c_int32, ctypes.c_int,
                                                 ctypes.c_int, _F64_3, ctypes.c_double, _ex]),
    "harpia_morph3d_batched": (ctypes.c_int, [ctypes.POINTER(harpia_crop), ctypes.c_int32, ctypes.c_int,
                                              ctypes.c_int, ctypes.c_int, _I32_3, _ex]),
    "harpia_gaussian3d_backward_batched": (ctypes.c_int, [ctypes.POINTER(harpia_crop), ctypes.c_int32, _F64_3,
                                                          _I32_3, _vp, _vp, ctypes.c_size_t, _ex]),
    "harpia_morph3d_forward_batched": (ctypes.c_int, [ctypes.POINTER(harpia_crop), ctypes.c_int32,
                                                      ctypes.c_int, ctypes.c_int, _I32_3, _vp,
                                                      ctypes.c_size_t, _ex]),
    "harpia_morph3d_backward_batched": (ctypes.c_int, [ctypes.POINTER(harpia_crop), ctypes.c_int32,
                                                       ctypes.c_int, ctypes.c_int, _I32_3, _vp,
                                                       ctypes.c_size_t, _ex]),
    "harpia_autotune_gaussian3d": (ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.c_int, _I64_3, _F64_3,
                                                  ctypes.c_double, ctypes.c_int32, _ex,
                                                  ctypes.POINTER(harpia_tune_report)]),
    "harpia_autotune_erode_dilate3d": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _I64_3, ctypes.c_int, _I32_3,
                                                      ctypes.c_double, ctypes.c_int32, _ex,
                                                      ctypes.POINTER(harpia_tune_report)]),
    "harpia_autotune_gauss_dilate_batched": (ctypes.c_int, [ctypes.POINTER(harpia_crop), ctypes.c_int32, _F64_3,
                                                            _I32_3, ctypes.c_int, _I32_3, _vp, ctypes.c_size_t,
                                                            ctypes.c_int32, _ex,
                                                            ctypes.POINTER(harpia_tune_report)]),
    "harpia_tune_clear": (ctypes.c_int, []),
    "harpia_tune_entries": (ctypes.c_int64, []),
    "harpia_tune_save": (ctypes.c_int, [ctypes.c_char_p]),
    "harpia_tune_load": (ctypes.c_int, [ctypes.c_char_p]),
}

_lib = None


def load():
    """Load libharpia.so (built by paper_2511_11890_amd/build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libharpia.so is not built (%s); run __graft_entry__.build() or "
                          "python paper_2511_11890_amd/build.py" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int):
    """Raise HarpiaError with the library's message for a failing status."""
    if status != HARPIA_OK:
        msg = load().harpia_last_error()
        raise HarpiaError(status, msg.decode() if msg else "")


def i64_3(v):
    return _I64_3(*[int(t) for t in v])


def i32_3(v):
    return _I32_3(*[int(t) for t in v])


def f64_3(v):
    return _F64_3(*[float(t) for t in v])


def crops(triples):
    """harpia_crop array from (in, out, aux) tensors (aux / out may be None)."""
    arr = (harpia_crop * len(triples))()
    for i, (a, b, c) in enumerate(triples):
        ref = a if a is not None else (b if b is not None else c)
        arr[i].in_ = a.data_ptr() if a is not None else None
        arr[i].out = b.data_ptr() if b is not None else None
        arr[i].aux = c.data_ptr() if c is not None else None
        arr[i].shape = i64_3(ref.shape)
    return arr


def make_exec(budget: int = 0, fraction: float = 0.0, chunk=(0, 0, 0), stream: int | None = None,
              flags: int = 0, stats: harpia_stats | None = None) -> harpia_exec:
    ex = harpia_exec()
    ex.device_budget_bytes = int(budget)
    ex.budget_fraction = float(fraction)
    ex.chunk = i64_3(chunk)
    ex.stream = stream
    ex.flags = int(flags)
    ex.stats = ctypes.pointer(stats) if stats is not None else None
    return ex
