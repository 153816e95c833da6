"""Chunked execution (Section III-D): volumes split into halo-padded chunks
under a device budget must give output bitwise equal to the resident run,
for z-slab and brick plans, from pageable and pinned host memory, and leave
no device memory behind (Section I, contribution 2; Section IV-C)."""
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2511_11890_amd as h
from paper_2511_11890_amd import phantoms
from tests.gpu_util import to_np64

pytestmark = pytest.mark.gpu

SHAPE = (70, 90, 150)


def _ops():
    """(name, fn(x, ex)) for every filter family on a u16 / f32 input."""
    return [
        ("gauss_s2", lambda x, ex: h.gaussian(x, 2.0, ex=ex)),
        ("gauss_s4", lambda x, ex: h.gaussian(x, 4.0, ex=ex)),
        ("gauss_aniso", lambda x, ex: h.gaussian(x, (1.0, 2.0, 1.5), ex=ex)),
        ("open_ball2", lambda x, ex: h.opening(x, "ball", 2, threshold=32768.0, ex=ex)),
        ("erode_ball3", lambda x, ex: h.erode(x, "ball", 3, ex=ex)),
        ("close_box1", lambda x, ex: h.closing(x, "box", 1, threshold=32768.0, ex=ex)),
    ]


@pytest.fixture(scope="module")
def vol_u16():
    return phantoms.porous_u16(SHAPE, seed=21)


@pytest.mark.parametrize("name,fn", _ops())
@pytest.mark.parametrize("chunk", [(0, 0, 0), (16, 40, 64), (13, 90, 150)])
def test_device_chunked_equals_resident(dev, vol_u16, name, fn, chunk):
    x = vol_u16.to(dev)
    ref = fn(x, None)
    got = fn(x, h.Exec(force_chunked=True, chunk=chunk, budget=64 << 20))
    torch.cuda.synchronize()
    assert torch.equal(ref, got), name


@pytest.mark.parametrize("name,fn", _ops())
@pytest.mark.parametrize("chunk,budget", [((0, 0, 0), 3 << 20), ((24, 32, 48), 16 << 20),
                                          ((70, 90, 150), 512 << 20)])
@pytest.mark.parametrize("mem", ["pageable", "pinned"])
def test_host_streamed_equals_resident(dev, vol_u16, name, fn, chunk, budget, mem):
    ref = fn(vol_u16.to(dev), None)
    x = vol_u16.pin_memory() if mem == "pinned" else vol_u16.numpy()
    st = h.harpia_stats()
    got = fn(x, h.Exec(budget=budget, chunk=chunk, stats=st))
    got_t = torch.from_numpy(got) if isinstance(got, np.ndarray) else got
    assert torch.equal(ref.cpu(), got_t), (name, chunk, mem)
    assert st.peak_device_bytes <= budget
    if chunk == (0, 0, 0) and budget < (8 << 20):
        assert st.n_chunks > 1
    assert st.bytes_d2h >= got_t.numel() * got_t.element_size()


def test_streamed_matches_oracle(dev):
    # independent of the resident path: the streamed result vs the oracle
    v = phantoms.porous((40, 50, 120), seed=22).numpy()
    st = h.harpia_stats()
    got = h.gaussian(v, 2.0, ex=h.Exec(budget=1 << 20, stats=st))
    assert st.n_chunks > 2
    v64 = v.astype(np.float64)
    want = oracle.gaussian3d(v64, 2.0, method="separable")
    scale = oracle.gaussian3d(np.abs(v64), 2.0, method="separable")
    assert np.all(np.abs(got.astype(np.float64) - want) <= 1e-5 * scale)


def test_budget_error_and_no_leak(dev, vol_u16):
    x = vol_u16.numpy()
    torch.cuda.synchronize()
    h.gaussian(x, 2.0, ex=h.Exec(budget=4 << 20))  # warm the runtime
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(10):
        h.gaussian(x, 2.0, ex=h.Exec(budget=4 << 20))
        h.opening(x, "ball", 2, threshold=32768.0, ex=h.Exec(budget=4 << 20))
    with pytest.raises(h.HarpiaError) as e:
        h.gaussian(x, 2.0, ex=h.Exec(budget=64 << 10))
    assert e.value.status == -3  # HARPIA_ERR_BUDGET
    free1 = torch.cuda.mem_get_info()[0]
    assert free1 >= free0  # nothing left behind (the runtime may release its own buffers meanwhile)


@pytest.mark.parametrize("at", [1, 2, 3])
def test_injected_allocation_failure_frees_everything(dev, vol_u16, at):
    x = vol_u16.numpy()
    h.gaussian(x, 2.0, ex=h.Exec(budget=4 << 20))
    free0 = torch.cuda.mem_get_info()[0]
    os.environ["HARPIA_TEST_FAIL_ALLOC_AT"] = str(at)
    try:
        with pytest.raises(h.HarpiaError) as e:
            h.gaussian(x, 2.0, ex=h.Exec(budget=4 << 20))  # arena, pinned in, pinned out
        assert e.value.status == -4  # HARPIA_ERR_OOM
    finally:
        del os.environ["HARPIA_TEST_FAIL_ALLOC_AT"]
    assert torch.cuda.mem_get_info()[0] >= free0  # nothing left behind
    got = h.gaussian(x, 2.0, ex=h.Exec(budget=4 << 20))  # still works afterwards
    assert got.shape == x.shape


def test_mixed_pointers_rejected(dev, vol_u16):
    x = vol_u16.to(dev)
    out = np.empty(SHAPE, np.float32)
    with pytest.raises(h.HarpiaError) as e:
        h.gaussian(x, 1.0, out=out)
    assert e.value.status == -1


def test_resident_no_device_memory_kept(dev):
    x = torch.from_numpy(phantoms.porous((64, 64, 64), seed=23).numpy()).to(dev)
    y = h.gaussian(x, 1.0)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(20):
        h.gaussian(x, 1.0, out=y)
        h.gaussian(x, (1.0, 0.5, 2.0), out=y)  # unfused: allocates and frees scratch
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] >= free0  # nothing left behind
