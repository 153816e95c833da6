"""Host-side tests of the C ABI: the library loads without a GPU, exports
every function include/harpia.h declares, validates arguments before any
device work, and plans chunks (Section III-D: a fixed fraction of free
memory, the deepest z-slab that fits with its padding) within the budget."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import paper_2511_11890_amd as h
from paper_2511_11890_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "harpia.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(harpia_\w+)\s*\(", text)))


def test_header_declares_the_core_calls():
    names = declared_functions()
    for n in ("harpia_gaussian3d", "harpia_erode3d", "harpia_dilate3d", "harpia_chunk_plan",
              "harpia_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol():
    assert set(declared_functions()) <= set(_lib.SIGNATURES)


def test_version_and_radius():
    assert h.version().startswith("harpia")
    assert h.gauss_radius(1.0) == 3
    assert h.gauss_radius(1.5) == 5
    assert h.gauss_radius(1.499) == 4
    assert h.gauss_radius(2.0) == 6
    assert h.gauss_radius(4.0) == 12
    assert h.gauss_radius(-1.0) == -1


def _status(fn):
    with pytest.raises(_lib.HarpiaError) as e:
        fn()
    return e.value.status


def test_validation_errors_before_device_work():
    a = np.zeros((4, 5, 6), np.float32)
    b = np.zeros((4, 5, 6), np.float32)
    assert _status(lambda: h.gaussian(a, 0.0)) == _lib.HARPIA_ERR_ARG
    assert _status(lambda: h.gaussian(a, float("nan"))) == _lib.HARPIA_ERR_ARG
    assert _status(lambda: h.gaussian(a, 1.0, truncate=-1.0)) == _lib.HARPIA_ERR_ARG
    assert _status(lambda: h.gaussian(a, 1.0, out=a)) == _lib.HARPIA_ERR_ALIAS
    assert _status(lambda: h.gaussian(a, 1.0, out=np.zeros((4, 5, 6), np.float16))) == _lib.HARPIA_ERR_DTYPE
    assert _status(lambda: h.gaussian(a, 30.0)) == _lib.HARPIA_ERR_UNSUPPORTED  # r = 90
    assert _status(lambda: h.erode(a, "ball", (1, 2, 2))) == _lib.HARPIA_ERR_ARG
    assert _status(lambda: h.erode(a, "box", -1)) == _lib.HARPIA_ERR_ARG
    assert _status(lambda: h.dilate(a, "box", 1, out=a)) == _lib.HARPIA_ERR_ALIAS
    del b


def test_raw_abi_null_and_shape_checks():
    lib = _lib.load()
    shape = _lib.i64_3((4, 4, 4))
    buf = (ctypes.c_float * 64)()
    out = (ctypes.c_float * 64)()
    st = lib.harpia_gaussian3d(None, _lib.HARPIA_F32, out, _lib.HARPIA_F32, shape, _lib.f64_3((1, 1, 1)),
                               3.0, 0, None)
    assert st == _lib.HARPIA_ERR_ARG
    assert b"NULL" in lib.harpia_last_error()
    st = lib.harpia_gaussian3d(buf, _lib.HARPIA_F32, out, _lib.HARPIA_F32, _lib.i64_3((0, 4, 4)),
                               _lib.f64_3((1, 1, 1)), 3.0, 0, None)
    assert st == _lib.HARPIA_ERR_ARG
    st = lib.harpia_gaussian3d(buf, 9, out, _lib.HARPIA_F32, shape, _lib.f64_3((1, 1, 1)), 3.0, 0, None)
    assert st == _lib.HARPIA_ERR_DTYPE
    st = lib.harpia_gaussian3d(buf, _lib.HARPIA_F32, out, _lib.HARPIA_F32, shape, _lib.f64_3((1, 1, 1)),
                               3.0, 7, None)
    assert st == _lib.HARPIA_ERR_ARG
    ops = (ctypes.c_int * 1)(5)
    st = lib.harpia_morph3d(buf, out, _lib.HARPIA_F32, shape, ops, 1, 0, _lib.i32_3((1, 1, 1)),
                            float("nan"), 0, None)
    assert st == _lib.HARPIA_ERR_ARG
    st = lib.harpia_morph3d(buf, out, _lib.HARPIA_F32, shape, ops, 0, 0, _lib.i32_3((1, 1, 1)),
                            float("nan"), 0, None)
    assert st == _lib.HARPIA_ERR_ARG


# ------------------------------------------------------------------ planner

def _tiles(p):
    """Core boxes of a plan, z slowest."""
    out = []
    for iz in range(p.grid[0]):
        for iy in range(p.grid[1]):
            for ix in range(p.grid[2]):
                lo = [iz * p.core[0], iy * p.core[1], ix * p.core[2]]
                hi = [min(p.shape[a], lo[a] + p.core[a]) for a in range(3)]
                out.append((lo, hi))
    return out


@pytest.mark.parametrize("shape,halo,budget,chunk", [
    ((100, 37, 53), (3, 3, 3), 1 << 20, (0, 0, 0)),
    ((64, 64, 64), (6, 6, 6), 8 << 20, (16, 24, 40)),
    ((2048, 2048, 2048), (6, 6, 6), 8 << 30, (512, 512, 512)),
    ((2048, 2048, 2048), (4, 4, 4), 8 << 30, (0, 0, 0)),
    ((7, 5, 3), (12, 12, 12), 1 << 20, (0, 0, 0)),
])
def test_plan_covers_volume_within_budget(shape, halo, budget, chunk):
    p = h.plan(shape, "u16", "f32", halo, budget=budget, chunk=chunk)
    assert list(p.shape) == list(shape)
    assert p.device_bytes <= budget
    assert p.n_buffers >= 1
    assert p.n_chunks == p.grid[0] * p.grid[1] * p.grid[2]
    assert list(p.halo) == list(halo)
    if chunk == (0, 0, 0):  # z-slabs
        assert p.core[1] == shape[1] and p.core[2] == shape[2]
    count = np.zeros(shape[:1] + (1, 1), np.int64) if max(shape) > 256 else np.zeros(shape, np.int64)
    if max(shape) <= 256:
        for lo, hi in _tiles(p):
            count[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] += 1
        assert np.all(count == 1)  # every voxel in exactly one core
    else:
        for a in range(3):
            assert p.grid[a] * p.core[a] >= shape[a] > (p.grid[a] - 1) * p.core[a]


def test_plan_z_slab_is_deepest_that_fits():
    shape, halo = (200, 64, 64), (2, 2, 2)
    budget = 4 << 20
    p = h.plan(shape, "f32", "f32", halo, budget=budget)
    # one more slice must not fit with the same number of buffer sets
    per_slice_in = 64 * 64 * 4
    need_next = p.n_buffers * ((p.core[0] + 1 + 4) * per_slice_in + (p.core[0] + 1) * per_slice_in)
    assert need_next > budget or p.core[0] == shape[0]


def test_plan_budget_errors():
    assert _status(lambda: h.plan((64, 1024, 1024), "f32", "f32", (4, 4, 4), budget=1 << 20)) == \
        _lib.HARPIA_ERR_BUDGET
    assert _status(lambda: h.plan((64, 64, 64), "f32", "f32", (4, 4, 4), budget=1 << 20,
                                  chunk=(64, 64, 64))) == _lib.HARPIA_ERR_BUDGET
    assert _status(lambda: h.plan((0, 64, 64), "f32", "f32", (4, 4, 4), budget=1 << 20)) == \
        _lib.HARPIA_ERR_ARG
    assert _status(lambda: h.plan((8, 8, 8), "f32", "f32", (-1, 0, 0), budget=1 << 20)) == \
        _lib.HARPIA_ERR_ARG


def test_plan_paper_config_brick_counts():
    # 2048^3 u16 -> f32, 8 GiB cap, 512^3 bricks, halo 6: 64 chunks; the
    # halo-padded input brick is 524^3 u16.
    p = h.plan((2048,) * 3, "u16", "f32", (6, 6, 6), budget=8 << 30, chunk=(512, 512, 512))
    assert p.n_chunks == 64
    per_set = math.ceil(524 ** 3 * 2 / 256) * 256 + 512 ** 3 * 4
    assert p.device_bytes == p.n_buffers * per_set


def _plain_host() -> bool:
    try:
        import torch
        return not torch.cuda.is_available()
    except Exception:
        return True


@pytest.mark.skipif(not _plain_host(), reason="the unclipped cap is the no-device case")
def test_budget_env_is_only_a_default(monkeypatch):
    # Section III-D, step 1: the caller's cap wins over the environment's
    # default; with no cap given, the environment's cap is used.
    monkeypatch.setenv("HARPIA_DEVICE_BUDGET", str(3 << 20))
    p = h.plan((64, 64, 64), "f32", "f32", (1, 1, 1), budget=5 << 20)
    assert p.budget_bytes == 5 << 20
    p = h.plan((64, 64, 64), "f32", "f32", (1, 1, 1))
    assert p.budget_bytes == 3 << 20
    monkeypatch.delenv("HARPIA_DEVICE_BUDGET")
    assert _status(lambda: h.plan((64, 64, 64), "f32", "f32", (1, 1, 1))) == _lib.HARPIA_ERR_ARG
