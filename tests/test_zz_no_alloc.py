"""The no-allocation Gaussian backward (harpia_gaussian3d_backward_noalloc)
through the raw C ABI: equal to harpia_gaussian3d_backward on two calls in a
row (the second on a smaller volume, so stale scratch from the first would
show), with device and host sigma-gradient destinations, under an injected
allocation failure (any device allocation would fail the call), and its
size limit."""
import ctypes
import os

import numpy as np
import pytest
import torch

import paper_2511_11890_amd as h
from paper_2511_11890_amd import _lib, phantoms

pytestmark = pytest.mark.gpu


def _call(fn, x, g, gi, shape, sigma, r, gs, flags=0):
    lib = _lib.load()
    return getattr(lib, fn)(
        x.data_ptr() if x is not None else None, _lib.HARPIA_F32, g.data_ptr(),
        gi.data_ptr() if gi is not None else None, _lib.i64_3(shape), _lib.f64_3((sigma,) * 3),
        _lib.i32_3((r,) * 3), gs, _lib.make_exec(stream=torch.cuda.current_stream().cuda_stream, flags=flags))


def _noalloc(*args, **kw):
    """The no-allocation call with the library's allocation hook armed: its
    first device or pinned allocation, if it made one, would fail."""
    os.environ["HARPIA_TEST_FAIL_ALLOC_AT"] = "1"
    try:
        return _call("harpia_gaussian3d_backward_noalloc", *args, **kw)
    finally:
        del os.environ["HARPIA_TEST_FAIL_ALLOC_AT"]


@pytest.mark.parametrize("sigma", [1.5, 4.0])
def test_noalloc_equals_allocating_backward(dev, sigma):
    r = h.gauss_radius(sigma)
    for k, shape in enumerate([(40, 70, 150), (17, 33, 61)]):
        x = phantoms.porous(shape, seed=80 + k).to(dev)
        g = phantoms.gaussian_noise(shape, seed=90 + k).to(dev)
        gi_a, gi_b = torch.empty_like(g), torch.empty_like(g)
        gs_a = torch.zeros(3, dtype=torch.float64, device=dev)
        gs_b = torch.full((3,), 7.0, dtype=torch.float64, device=dev)
        assert _noalloc(x, g, gi_b, shape, sigma, r, gs_b.data_ptr()) == 0, _lib.load().harpia_last_error()
        assert _call("harpia_gaussian3d_backward", x, g, gi_a, shape, sigma, r, gs_a.data_ptr()) == 0
        torch.cuda.synchronize()
        assert torch.equal(gi_a, gi_b), shape
        assert torch.equal(gs_a, gs_b), (shape, gs_a, gs_b)
        # host destination and the summed isotropic gradient
        host = np.full(3, 7.0)
        assert _noalloc(x, g, None, shape, sigma, r, host.ctypes.data, _lib.HARPIA_F_SIGMA_SUM) == 0, \
            _lib.load().harpia_last_error()
        assert host[1] == 7.0 and host[2] == 7.0
        _, gsum = h.gaussian_backward(x, g, sigma, (r,) * 3, grad_in=False, sigma_sum=True)
        assert host[0] == float(gsum[0])


def test_noalloc_limits(dev):
    x = torch.zeros((8, 9, 10), device=dev)
    gs = torch.zeros(3, dtype=torch.float64, device=dev)
    # unequal radii need the unfused passes, which need scratch volumes
    lib = _lib.load()
    st = lib.harpia_gaussian3d_backward_noalloc(
        x.data_ptr(), _lib.HARPIA_F32, x.data_ptr(), None, _lib.i64_3(x.shape), _lib.f64_3((1.0, 2.0, 1.0)),
        _lib.i32_3((3, 6, 3)), gs.data_ptr(), _lib.make_exec(stream=torch.cuda.current_stream().cuda_stream))
    assert st == _lib.HARPIA_ERR_UNSUPPORTED
    # a volume whose partials exceed the fixed scratch (only its shape is
    # checked: the call fails before any launch)
    big = (4096, 4096, 4096)
    st = lib.harpia_gaussian3d_backward_noalloc(
        x.data_ptr(), _lib.HARPIA_F32, x.data_ptr(), None, _lib.i64_3(big), _lib.f64_3((1.0,) * 3),
        _lib.i32_3((3,) * 3), gs.data_ptr(), _lib.make_exec(stream=torch.cuda.current_stream().cuda_stream))
    assert st == _lib.HARPIA_ERR_ARG
    assert b"scratch" in lib.harpia_last_error()
