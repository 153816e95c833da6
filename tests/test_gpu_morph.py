"""GPU parity of erosion / dilation / opening / closing against the FP64
brute-force oracle (Section III-C label-editing morphology): bit-exact for
every dtype, grayscale and binary, box and ball elements."""
import numpy as np
import pytest
import torch

import oracle
import paper_2511_11890_amd as h
from paper_2511_11890_amd import phantoms
from tests.gpu_util import sample_points, to_np64, window_of

pytestmark = pytest.mark.gpu

# several 64 x 16 grayscale tiles and 256 x 16 binary tiles, ragged tails
SHAPE = (23, 37, 300)


def _gray(shape, dtype, seed):
    v = phantoms.porous(shape, seed=seed)
    if dtype == torch.float32:
        return v
    if dtype == torch.uint16:
        return phantoms.porous_u16(shape, seed=seed)
    if dtype == torch.uint8:
        return (phantoms.porous_u16(shape, seed=seed).to(torch.int32) >> 8).to(torch.uint8)
    return torch.clamp(v, 0, 1).to(dtype)


DTYPES = [torch.float32, torch.uint16, torch.uint8, torch.float16, torch.bfloat16]
ELEMENTS = [("box", 1), ("box", 2), ("box", 3), ("ball", 1), ("ball", 2), ("ball", 3), ("ball", 4)]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("se,r", ELEMENTS)
def test_gray_erode_dilate_bit_exact(dev, dtype, se, r):
    v = _gray(SHAPE, dtype, seed=11)
    vd = v.to(dev)
    print("gray", dtype, se, r, flush=True)
    e = h.erode(vd, se, r)
    d = h.dilate(vd, se, r)
    e2, d2 = h.erode_dilate(vd, se, r)
    torch.cuda.synchronize()
    v64 = to_np64(v)
    we = oracle.erode3d(v64, se, r)
    wd = oracle.dilate3d(v64, se, r)
    assert e.dtype == dtype and d.dtype == dtype
    np.testing.assert_array_equal(to_np64(e), we)
    np.testing.assert_array_equal(to_np64(d), wd)
    np.testing.assert_array_equal(to_np64(e2), we)
    np.testing.assert_array_equal(to_np64(d2), wd)


def _order_keys(a):
    """float32 -> int32 keys whose order is the IEEE 754 totalOrder."""
    b = a.view(np.int32).astype(np.int64)
    return np.where(b < 0, b ^ 0x7FFFFFFF, b)


def _box_extremum(keys, r, fn):
    # brute force over the box, offsets outside the volume skipped
    nz, ny, nx = keys.shape
    out = np.empty_like(keys)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                out[z, y, x] = fn(keys[max(0, z - r[0]):z + r[0] + 1, max(0, y - r[1]):y + r[1] + 1,
                                       max(0, x - r[2]):x + r[2] + 1])
    return out


@pytest.mark.parametrize("r", [(1, 1, 1), (2, 2, 2), (1, 2, 0)])
def test_gray_total_order_of_zeros_and_nans(dev, r):
    # the header's rule for values float comparison leaves open: -0 < +0,
    # and NaNs beyond the infinities on the side of their sign; fast
    # (isotropic) and generic (anisotropic) kernels, single and paired
    rng = np.random.default_rng(41)
    v = rng.standard_normal((7, 12, 70)).astype(np.float32)
    flat = v.reshape(-1)
    idx = rng.permutation(flat.size)
    flat[idx[:40]] = 0.0
    flat[idx[40:80]] = -0.0
    flat[idx[80:86]] = np.float32(np.inf)
    flat[idx[86:92]] = np.float32(-np.inf)
    nan = np.array([0x7FC00000, 0xFFC00000], dtype=np.uint32).view(np.float32)
    flat[idx[92:95]] = nan[0]
    flat[idx[95:98]] = nan[1]
    keys = _order_keys(v)
    want_e = _box_extremum(keys, r, np.min)
    want_d = _box_extremum(keys, r, np.max)
    vd = torch.from_numpy(v).to(dev)
    e, d = h.erode(vd, "box", r), h.dilate(vd, "box", r)
    e2, d2 = h.erode_dilate(vd, "box", r)
    torch.cuda.synchronize()
    for got, want in ((e, want_e), (d, want_d), (e2, want_e), (d2, want_d)):
        np.testing.assert_array_equal(_order_keys(got.cpu().numpy()), want)


@pytest.mark.parametrize("r", [(1, 2, 3), (0, 0, 2), (3, 0, 1), (0, 0, 0)])
def test_gray_anisotropic_box_generic_path(dev, r):
    v = _gray((19, 29, 70), torch.float32, seed=12)
    e = h.erode(v.to(dev), "box", r)
    d = h.dilate(v.to(dev), "box", r)
    torch.cuda.synchronize()
    v64 = to_np64(v)
    np.testing.assert_array_equal(to_np64(e), oracle.erode3d(v64, "box", r))
    np.testing.assert_array_equal(to_np64(d), oracle.dilate3d(v64, "box", r))


def test_gray_large_ball_generic_path(dev):
    v = _gray((17, 21, 40), torch.uint16, seed=13)
    e, d = h.erode_dilate(v.to(dev), "ball", 6)
    torch.cuda.synchronize()
    v64 = to_np64(v)
    np.testing.assert_array_equal(to_np64(e), oracle.erode3d(v64, "ball", 6))
    np.testing.assert_array_equal(to_np64(d), oracle.dilate3d(v64, "ball", 6))


@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 3, 4), (1, 1, 300), (300, 1, 2), (5, 64, 1)])
@pytest.mark.parametrize("se,r", [("box", 2), ("ball", 3)])
def test_gray_degenerate_shapes(dev, shape, se, r):
    v = _gray(shape, torch.float32, seed=14)
    e, d = h.erode_dilate(v.to(dev), se, r)
    torch.cuda.synchronize()
    v64 = to_np64(v)
    np.testing.assert_array_equal(to_np64(e), oracle.erode3d(v64, se, r))
    np.testing.assert_array_equal(to_np64(d), oracle.dilate3d(v64, se, r))


def _binary_case(kind, shape, seed):
    """(input tensor, threshold or None, binary flag, oracle 0/1 volume)."""
    if kind == "f32":
        v = phantoms.blobs(seed=seed, shape=shape)
        t = torch.from_numpy(v)
        return t, 0.5, False, oracle.threshold(v.astype(np.float64), 0.5)
    if kind == "u16":
        t = phantoms.porous_u16(shape, seed=seed)
        return t, 32768.0, False, oracle.threshold(to_np64(t), 32768.0)
    if kind == "u8flag":
        b = (phantoms.porous(shape, seed=seed) > 0.5).to(torch.uint8)
        return b, None, True, to_np64(b)
    if kind == "u8thr":
        t = (phantoms.porous_u16(shape, seed=seed).to(torch.int32) >> 8).to(torch.uint8)
        return t, 127.0, False, oracle.threshold(to_np64(t), 127.0)
    if kind == "f32_nonrep":  # threshold not representable in float32
        v = phantoms.porous(shape, seed=seed)
        thr = 0.5 + 1e-12
        return v, thr, False, oracle.threshold(to_np64(v), thr)
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["f32", "u16", "u8flag", "f32_nonrep"])
@pytest.mark.parametrize("se,r", ELEMENTS)
def test_binary_erode_dilate_bit_exact(dev, kind, se, r):
    t, thr, flag, b = _binary_case(kind, SHAPE, seed=15)
    td = t.to(dev)
    print("binary", kind, se, r, flush=True)
    e = h.erode(td, se, r, threshold=thr, binary=flag)
    d = h.dilate(td, se, r, threshold=thr, binary=flag)
    e2, d2 = h.erode_dilate(td, se, r, threshold=thr, binary=flag)
    torch.cuda.synchronize()
    assert e.dtype == torch.uint8
    we, wd = oracle.erode3d(b, se, r), oracle.dilate3d(b, se, r)
    for got, want in ((e, we), (d, wd), (e2, we), (d2, wd)):
        np.testing.assert_array_equal(to_np64(got), want)


@pytest.mark.parametrize("kind", ["u16", "u8flag", "u8thr"])
@pytest.mark.parametrize("nx", [336, 208])
@pytest.mark.parametrize("se,r", [("box", 1), ("ball", 2), ("box", 3), ("ball", 4)])
def test_binary_aligned_rows_bit_exact(dev, kind, nx, se, r):
    """Rows that are whole multiples of 16 bytes: strips whose 64-voxel core
    lies in the read window load it in 16-byte pieces, while the last,
    partial strip (nx mod 64 = 16) and the halo groups at the x faces take
    the per-group loads."""
    t, thr, flag, b = _binary_case(kind, (13, 70, nx), seed=19)
    td = t.to(dev)
    print("binary aligned", kind, nx, se, r, flush=True)
    e = h.erode(td, se, r, threshold=thr, binary=flag)
    e2, d2 = h.erode_dilate(td, se, r, threshold=thr, binary=flag)
    torch.cuda.synchronize()
    we, wd = oracle.erode3d(b, se, r), oracle.dilate3d(b, se, r)
    for got, want in ((e, we), (e2, we), (d2, wd)):
        np.testing.assert_array_equal(to_np64(got), want)


def test_binary_threshold_ties_u16(dev):
    # voxels equal to the threshold are background (strict >)
    v = torch.full((9, 20, 300), 32768, dtype=torch.uint16)
    v[4, 10, 100] = 32769
    d = h.dilate(v.to(dev), "box", 1, threshold=32768.0)
    torch.cuda.synchronize()
    assert int(d.sum().item()) == 27


@pytest.mark.parametrize("se,r", [("box", 1), ("ball", 2), ("ball", 3)])
@pytest.mark.parametrize("chain", [["erode", "dilate"], ["dilate", "erode"], ["erode", "erode", "dilate"]])
def test_binary_chains(dev, se, r, chain):
    t, thr, flag, b = _binary_case("u16", (31, 41, 290), seed=16)
    got = h.morph(t.to(dev), chain, se, r, threshold=thr)
    torch.cuda.synchronize()
    want = b
    for op in chain:
        want = oracle.morph3d(want, op, se, r)
    np.testing.assert_array_equal(to_np64(got), want)


@pytest.mark.parametrize("se,r", [("box", 2), ("ball", 2)])
def test_gray_opening_closing(dev, se, r):
    v = _gray((25, 33, 100), torch.float32, seed=17)
    o = h.opening(v.to(dev), se, r)
    c = h.closing(v.to(dev), se, r)
    torch.cuda.synchronize()
    v64 = to_np64(v)
    np.testing.assert_array_equal(to_np64(o), oracle.opening3d(v64, se, r))
    np.testing.assert_array_equal(to_np64(c), oracle.closing3d(v64, se, r))


def test_morph_full_size_sampled(dev):
    """1024^3 float32 porous phantom, grayscale erosion + dilation with the
    ball of radius 3 (the resident workload): sampled voxels vs the oracle."""
    shape = (1024, 1024, 1024)
    v = phantoms.porous(shape, seed=0, device=dev)
    e, d = h.erode_dilate(v, "ball", 3)
    torch.cuda.synchronize()
    pts = sample_points(shape, 128, seed=3)
    idx = torch.tensor(pts, device=dev)
    ge = e[idx[:, 0], idx[:, 1], idx[:, 2]].double().cpu().numpy()
    gd = d[idx[:, 0], idx[:, 1], idx[:, 2]].double().cpu().numpy()
    for p, a, b in zip(pts, ge, gd):
        win = window_of(v, p, 3)
        assert a == oracle.erode3d(win, "ball", 3)[3, 3, 3], p
        assert b == oracle.dilate3d(win, "ball", 3)[3, 3, 3], p
    # order property over the whole volume: erosion <= v <= dilation
    assert bool(torch.all(e <= v)) and bool(torch.all(v <= d))
