"""GPU parity of the mean (box) filter and unsharp masking against the FP64
oracle (Section III-C filtering suite).

Mean: a positive-weight stencil, so the FP32 bound is the Gaussian's,
|gpu - oracle| <= 1e-5 * M(|v|) with M the mean filter; 16-bit storage
within 2u * M(|v|).
Unsharp, out = (1 + a) v - a G v: the Gaussian's error enters scaled by |a|
and the combination adds a few FP32 roundings of (1 + |a|) |v|, so
|gpu - oracle| <= 1e-5 * ((1 + |a|) |v| + |a| G(|v|)); 16-bit within
2u times the same scale."""
import numpy as np
import pytest
import torch

import oracle
import paper_2511_11890_amd as h
from paper_2511_11890_amd import phantoms
from tests.gpu_util import (FP32_GAUSS_TOL, U_BF16, U_F16, assert_gauss_close, gauss_scale, sample_points, to_np64,
                            window_of)

pytestmark = pytest.mark.gpu

# several 64 x 16 tiles with ragged tails in x and y
SHAPE = (37, 45, 150)


def _mean_scale(v64, r):
    return oracle.mean3d(np.abs(v64), r, method="separable")


def _unsharp_scale(v64, sigma, a):
    return (1 + abs(a)) * np.abs(v64) + abs(a) * gauss_scale(v64, sigma)


@pytest.mark.parametrize("r", [1, 2, 3, 12, (1, 2, 3), (0, 1, 2)])
def test_mean_f32(dev, r):
    v = phantoms.porous(SHAPE, seed=90).numpy()
    print("mean f32", SHAPE, r, flush=True)
    got = h.mean(torch.from_numpy(v).to(dev), r)
    torch.cuda.synchronize()
    v64 = v.astype(np.float64)
    want = oracle.mean3d(v64, r, method="separable")
    assert_gauss_close(to_np64(got), want, _mean_scale(v64, r), FP32_GAUSS_TOL, "r=%s" % (r,))


def test_mean_direct_form_and_degenerate(dev):
    for shape, r in (((9, 20, 70), 2), ((1, 1, 200), 3), ((3, 5, 7), 4), ((1, 1, 1), 1)):
        v = phantoms.gaussian_noise(shape, seed=91).numpy()
        got = h.mean(torch.from_numpy(v).to(dev), r)
        torch.cuda.synchronize()
        v64 = v.astype(np.float64)
        want = oracle.mean3d(v64, r, method="direct")
        assert_gauss_close(to_np64(got), want, _mean_scale(v64, r), FP32_GAUSS_TOL, str(shape))


@pytest.mark.parametrize("dtype,u", [(torch.bfloat16, U_BF16), (torch.float16, U_F16)])
def test_mean_16bit(dev, dtype, u):
    unq, v = phantoms.porous_16bit(SHAPE, dtype=dtype, seed=92)
    got = h.mean(v.to(dev), 2)
    assert got.dtype == dtype
    torch.cuda.synchronize()
    v_unq = unq.numpy().astype(np.float64)
    want = oracle.mean3d(v_unq, 2, method="separable")
    assert_gauss_close(to_np64(got), want, _mean_scale(v_unq, 2), 2 * u, "16-bit")


def test_mean_u16_to_f32_and_chunked(dev):
    v = phantoms.porous_u16(SHAPE, seed=93)
    res = h.mean(v.to(dev), 2)
    torch.cuda.synchronize()
    v64 = to_np64(v)
    assert_gauss_close(to_np64(res), oracle.mean3d(v64, 2, method="separable"), _mean_scale(v64, 2),
                       FP32_GAUSS_TOL, "u16")
    chunked = h.mean(v.to(dev), 2, ex=h.Exec(force_chunked=True, chunk=(8, 16, 64), budget=64 << 20))
    host = h.mean(v.pin_memory(), 2, ex=h.Exec(budget=8 << 20))
    torch.cuda.synchronize()
    assert torch.equal(chunked, res)
    assert torch.equal(host, res.cpu())


@pytest.mark.parametrize("sigma,amount", [(1.0, 0.5), (2.0, 1.5), (1.5, -0.5), (4.0, 1.0)])
def test_unsharp_f32(dev, sigma, amount):
    v = phantoms.porous(SHAPE, seed=94).numpy()
    print("unsharp f32", SHAPE, sigma, amount, flush=True)
    got = h.unsharp(torch.from_numpy(v).to(dev), sigma, amount)
    torch.cuda.synchronize()
    v64 = v.astype(np.float64)
    want = oracle.unsharp3d(v64, sigma, amount)
    assert_gauss_close(to_np64(got), want, _unsharp_scale(v64, sigma, amount), FP32_GAUSS_TOL,
                       "sigma=%g a=%g" % (sigma, amount))


def test_unsharp_zero_amount_is_identity_and_degenerate(dev):
    v = phantoms.gaussian_noise((9, 20, 70), seed=95)
    got = h.unsharp(v.to(dev), 2.0, 0.0)
    torch.cuda.synchronize()
    assert torch.equal(got.cpu(), v)
    for shape in ((1, 1, 200), (3, 5, 7), (1, 1, 1)):
        w = phantoms.gaussian_noise(shape, seed=96).numpy()
        got = h.unsharp(torch.from_numpy(w).to(dev), 2.0, 1.0)
        torch.cuda.synchronize()
        w64 = w.astype(np.float64)
        assert_gauss_close(to_np64(got), oracle.unsharp3d(w64, 2.0, 1.0), _unsharp_scale(w64, 2.0, 1.0),
                           FP32_GAUSS_TOL, str(shape))


@pytest.mark.parametrize("dtype,u", [(torch.bfloat16, U_BF16), (torch.float16, U_F16)])
def test_unsharp_16bit(dev, dtype, u):
    unq, v = phantoms.porous_16bit(SHAPE, dtype=dtype, seed=97)
    got = h.unsharp(v.to(dev), 1.0, 1.0)
    assert got.dtype == dtype
    torch.cuda.synchronize()
    v_unq = unq.numpy().astype(np.float64)
    want = oracle.unsharp3d(v_unq, 1.0, 1.0)
    assert_gauss_close(to_np64(got), want, _unsharp_scale(v_unq, 1.0, 1.0), 2 * u, "16-bit")


def test_unsharp_chunked_equals_resident(dev):
    v = phantoms.porous_u16(SHAPE, seed=98)
    res = h.unsharp(v.to(dev), 2.0, 0.8)
    dev_chunked = h.unsharp(v.to(dev), 2.0, 0.8, ex=h.Exec(force_chunked=True, chunk=(8, 16, 64), budget=64 << 20))
    host = h.unsharp(v.pin_memory(), 2.0, 0.8, ex=h.Exec(budget=8 << 20))
    torch.cuda.synchronize()
    assert torch.equal(dev_chunked, res)
    assert torch.equal(host, res.cpu())
    v64 = to_np64(v)
    assert_gauss_close(to_np64(res), oracle.unsharp3d(v64, 2.0, 0.8), _unsharp_scale(v64, 2.0, 0.8),
                       FP32_GAUSS_TOL, "u16")


def test_unsharp_limits(dev):
    v = torch.zeros((8, 9, 10), device=dev)
    with pytest.raises(h.HarpiaError):
        h.unsharp(v, (1.0, 2.0, 1.0), 1.0)  # unequal radii
    with pytest.raises(h.HarpiaError):
        h.unsharp(v, 5.0, 1.0)  # radius 15 > 12
    with pytest.raises(h.HarpiaError):
        h.unsharp(v, 1.0, float("inf"))
    with pytest.raises(h.HarpiaError):
        h.mean(v, -1)


# ------------------------------------------------------- Sobel / Prewitt
# Each axis response errs by at most eps * (|taps| * |v|), so the magnitude
# errs by at most eps * sqrt(sum_a (|taps_a| * |v|)^2).

def _edge_scale(v64, kind):
    sm = np.array([1.0, 2.0, 1.0]) if kind == "sobel" else np.ones(3)
    d = np.array([1.0, 0.0, 1.0])
    av = np.abs(v64)
    s2 = 0.0
    for a in range(3):
        s2 = s2 + oracle.conv3d(av, *[d if b == a else sm for b in range(3)], method="separable") ** 2
    return np.sqrt(s2)


@pytest.mark.parametrize("kind", ["sobel", "prewitt"])
def test_edge_f32(dev, kind):
    v = phantoms.porous(SHAPE, seed=99).numpy()
    print("edge f32", SHAPE, kind, flush=True)
    got = h.edge(torch.from_numpy(v).to(dev), kind)
    torch.cuda.synchronize()
    v64 = v.astype(np.float64)
    assert_gauss_close(to_np64(got), oracle.edge3d(v64, kind), _edge_scale(v64, kind), FP32_GAUSS_TOL, kind)


@pytest.mark.parametrize("shape", [(1, 1, 200), (3, 5, 7), (1, 1, 1), (2, 70, 1), (70, 1, 2), (5, 16, 64)])
def test_edge_degenerate_shapes(dev, shape):
    v = phantoms.gaussian_noise(shape, seed=100).numpy()
    got = h.edge(torch.from_numpy(v).to(dev), "sobel")
    torch.cuda.synchronize()
    v64 = v.astype(np.float64)
    assert_gauss_close(to_np64(got), oracle.edge3d(v64, "sobel"), _edge_scale(v64, "sobel"), FP32_GAUSS_TOL,
                       str(shape))


@pytest.mark.parametrize("dtype,u", [(torch.bfloat16, U_BF16), (torch.float16, U_F16)])
def test_edge_16bit(dev, dtype, u):
    unq, v = phantoms.porous_16bit(SHAPE, dtype=dtype, seed=101)
    got = h.edge(v.to(dev), "sobel")
    assert got.dtype == dtype
    torch.cuda.synchronize()
    v_unq = unq.numpy().astype(np.float64)
    assert_gauss_close(to_np64(got), oracle.edge3d(v_unq, "sobel"), _edge_scale(v_unq, "sobel"), 2 * u, "16-bit")


def test_edge_u16_chunked_equals_resident(dev):
    v = phantoms.porous_u16(SHAPE, seed=102)
    res = h.edge(v.to(dev), "prewitt")
    dev_chunked = h.edge(v.to(dev), "prewitt", ex=h.Exec(force_chunked=True, chunk=(8, 16, 64), budget=64 << 20))
    host = h.edge(v.pin_memory(), "prewitt", ex=h.Exec(budget=8 << 20))
    torch.cuda.synchronize()
    assert torch.equal(dev_chunked, res)
    assert torch.equal(host, res.cpu())
    v64 = to_np64(v)
    assert_gauss_close(to_np64(res), oracle.edge3d(v64, "prewitt"), _edge_scale(v64, "prewitt"), FP32_GAUSS_TOL,
                       "u16")


# ----------------------------------------------------------------- Hessian
# Component ab errs by at most 1e-5 * (|c_z| x |c_y| x |c_x|) * |v| (the
# separable correlation with the absolute taps).

def _hess_scale(v64, sigma):
    s = (sigma,) * 3 if np.ndim(sigma) == 0 else tuple(sigma)
    r = [oracle.gauss_radius(si) for si in s]
    out = []
    for a, b in oracle.HESSIAN_PAIRS:
        order = [0, 0, 0]
        order[a] += 1
        order[b] += 1
        taps = [np.abs(oracle.gauss_deriv_taps(s[i], r[i], order[i])) for i in range(3)]
        out.append(oracle.conv3d(np.abs(v64), *taps, method="separable"))
    return np.stack(out)


@pytest.mark.parametrize("sigma", [1.0, 2.0, (1.0, 1.5, 0.8)])
def test_hessian_f32(dev, sigma):
    v = phantoms.porous(SHAPE, seed=103).numpy()
    print("hessian f32", SHAPE, sigma, flush=True)
    got = h.hessian(torch.from_numpy(v).to(dev), sigma)
    torch.cuda.synchronize()
    assert got.shape == (6,) + SHAPE
    v64 = v.astype(np.float64)
    assert_gauss_close(to_np64(got), oracle.hessian3d(v64, sigma), _hess_scale(v64, sigma), FP32_GAUSS_TOL,
                       "sigma=%s" % (sigma,))


def test_hessian_u16_and_chunked(dev):
    # u16 input: odd components take the unfused passes
    v = phantoms.porous_u16((20, 33, 70), seed=104)
    res = h.hessian(v.to(dev), 1.0)
    host = h.hessian(v.pin_memory(), 1.0, ex=h.Exec(budget=4 << 20))
    torch.cuda.synchronize()
    v64 = to_np64(v)
    assert_gauss_close(to_np64(res), oracle.hessian3d(v64, 1.0), _hess_scale(v64, 1.0), FP32_GAUSS_TOL, "u16")
    assert torch.equal(host, res.cpu())
    x = torch.from_numpy(phantoms.porous((20, 33, 70), seed=105).numpy()).to(dev)
    a = h.hessian(x, 1.5)
    b = h.hessian(x, 1.5, ex=h.Exec(force_chunked=True, chunk=(8, 16, 64), budget=64 << 20))
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("sigma", [0.4, 0.7, 1.0, 1.3, (1.0, 0.9, 1.1)])
def test_hessian_two_pass_equals_six_passes(dev, sigma):
    # device-resident float32 with radii <= 4 runs two three-component
    # passes; the chunked device path runs the six one-component passes: the
    # per-voxel arithmetic is the same sequence, so the results are equal
    x = torch.from_numpy(phantoms.porous((23, 70, 150), seed=106).numpy()).to(dev)
    a = h.hessian(x, sigma)
    b = h.hessian(x, sigma, ex=h.Exec(force_chunked=True, chunk=(0, 0, 0), budget=1 << 30))
    torch.cuda.synchronize()
    assert torch.equal(a, b)


# -------------------------------------------------------- local thresholds
# The decision v > T is taken in FP32 on the GPU and in FP64 by the oracle:
# the two must agree wherever |v - T| exceeds the FP32 error bound of T
# (from the bounds of the mean m and of s = sqrt(q - m^2)), and that band
# must hold few voxels.

def _thr_band(v64, method, r, sigma, k, R, c):
    av = np.abs(v64)
    if method == "gaussian":
        return 2e-5 * (gauss_scale(v64, sigma) + abs(c)) + 1e-30
    m_scale = oracle.mean3d(av, r, method="separable")
    dm = 2e-5 * (m_scale + abs(c))
    if method == "mean":
        return dm + 1e-30
    q_scale = oracle.mean3d(av * av, r, method="separable")
    m = oracle.mean3d(v64, r, method="separable")
    var = np.maximum(oracle.mean3d(v64 * v64, r, method="separable") - m * m, 0)
    s = np.sqrt(var)
    dvar = 4e-5 * (q_scale + m_scale * m_scale)
    ds = np.where(s > np.sqrt(dvar), dvar / (2 * np.maximum(s, 1e-300)), np.sqrt(dvar))
    if method == "niblack":
        return dm + abs(k) * ds
    return np.abs(1 + k * (s / R - 1)) * dm + np.abs(m * k / R) * ds


@pytest.mark.parametrize("method,r,k", [("mean", 2, 0.0), ("gaussian", 0, 0.0), ("niblack", 2, -0.2),
                                        ("sauvola", 3, 0.5), ("niblack", 6, 0.3), ("mean", 12, 0.0)])
@pytest.mark.parametrize("dtype", ["f32", "u16", "u8"])
def test_local_threshold(dev, method, r, k, dtype):
    if dtype == "f32":
        v = phantoms.porous(SHAPE, seed=106)
    else:
        v = phantoms.porous_u16(SHAPE, seed=106)
        if dtype == "u8":
            v = (v.to(torch.int32) >> 8).to(torch.uint8)
    R = {"f32": 0.5, "u16": 32768.0, "u8": 128.0}[dtype]
    c = {"f32": 0.01, "u16": 300.0, "u8": 1.0}[dtype] if method in ("mean", "gaussian") else 0.0
    print("threshold", method, r, dtype, flush=True)
    got = h.local_threshold(v.to(dev), method, radius=r, sigma=1.5, k=k, r_param=R, offset=c)
    torch.cuda.synchronize()
    assert got.dtype == torch.uint8
    v64 = to_np64(v)
    want, t = oracle.local_threshold3d(v64, method, radius=r, sigma=1.5, k=k, r_param=R, offset=c, return_t=True)
    band = np.abs(v64 - t) <= _thr_band(v64, method, r, 1.5, k, R, c)
    g = got.cpu().numpy()
    bad = (g != want) & ~band
    assert not bad.any(), "%d decisions differ outside the FP32 band" % int(bad.sum())
    assert band.mean() < 0.02, band.mean()


def test_local_threshold_chunked_and_limits(dev):
    v = phantoms.porous_u16(SHAPE, seed=107)
    res = h.local_threshold(v.to(dev), "sauvola", radius=2, k=0.3, r_param=32768.0)
    chunked = h.local_threshold(v.to(dev), "sauvola", radius=2, k=0.3, r_param=32768.0,
                                ex=h.Exec(force_chunked=True, chunk=(8, 16, 64), budget=64 << 20))
    host = h.local_threshold(v.pin_memory(), "sauvola", radius=2, k=0.3, r_param=32768.0, ex=h.Exec(budget=8 << 20))
    torch.cuda.synchronize()
    assert torch.equal(chunked, res)
    assert torch.equal(host, res.cpu())
    x = torch.zeros((8, 9, 10), device=dev)
    with pytest.raises(h.HarpiaError):
        h.local_threshold(x, "niblack", radius=7)
    with pytest.raises(h.HarpiaError):
        h.local_threshold(x.to(torch.bfloat16), "mean", radius=1)
    with pytest.raises(h.HarpiaError):
        h.local_threshold(x, "sauvola", radius=1, r_param=0.0)


# -------------------------------------------------------------------- Otsu
# The split is decided in FP64 from exact integer sums on both sides: the
# threshold and the binary volume must equal the oracle's exactly.

@pytest.mark.parametrize("dtype", ["u8", "u16"])
@pytest.mark.parametrize("shape", [SHAPE, (1, 1, 777), (64, 64, 64)])
def test_otsu(dev, dtype, shape):
    v = phantoms.porous_u16(shape, seed=108)
    nb = 65536
    if dtype == "u8":
        v = (v.to(torch.int32) >> 8).to(torch.uint8)
        nb = 256
    print("otsu", dtype, shape, flush=True)
    out, k = h.otsu(v.to(dev))
    torch.cuda.synchronize()
    v64 = v.to(torch.int64).numpy()
    assert k == oracle.otsu_threshold(v64, nb)
    np.testing.assert_array_equal(out.cpu().numpy(), oracle.otsu3d(v64, nb))


@pytest.mark.parametrize("dtype", ["u8", "u16"])
def test_otsu_unaligned_and_large(dev, dtype):
    # a view that starts 3 elements into its storage (unaligned head and tail,
    # element-wise binarisation), and a 128^3 volume (many segments, the
    # concentrated two-phase histogram)
    nb = 256 if dtype == "u8" else 65536
    for shape, off in [((13, 17, 61), 3), ((128, 128, 128), 0)]:
        n = int(np.prod(shape))
        flat = phantoms.porous_u16((1, 1, n + off), seed=109).flatten()
        if dtype == "u8":
            flat = (flat.to(torch.int32) >> 8).to(torch.uint8)
        g = flat.to(dev)
        v = g[off:off + n].view(shape)
        assert off == 0 or v.data_ptr() % 16 != 0
        print("otsu", dtype, shape, off, flush=True)
        out, k = h.otsu(v)
        torch.cuda.synchronize()
        v64 = flat[off:off + n].view(shape).to(torch.int64).numpy()
        assert k == oracle.otsu_threshold(v64, nb)
        np.testing.assert_array_equal(out.cpu().numpy(), oracle.otsu3d(v64, nb))


def test_otsu_degenerate(dev):
    c = torch.full((5, 6, 7), 9, dtype=torch.uint8, device=dev)
    out, k = h.otsu(c)
    torch.cuda.synchronize()
    assert k == -1 and bool(out.all())
    two = torch.tensor([3, 3, 3, 10, 10], dtype=torch.uint8, device=dev).reshape(1, 1, 5)
    out, k = h.otsu(two)
    torch.cuda.synchronize()
    assert k == 3 and out.cpu().flatten().tolist() == [0, 0, 0, 1, 1]
    none, k2 = h.otsu(two, binarize=False)
    assert none is None and k2 == 3
    with pytest.raises(h.HarpiaError):
        h.otsu(torch.zeros((4, 4, 4), device=dev))  # float32: not an integer volume


# ------------------------------------------------- full size (1024^3, the
# filters workload's shapes and launch configuration): sampled voxels, each
# against the oracle on its reflected neighbourhood.

@pytest.fixture(scope="module")
def big_f32(dev):
    return phantoms.porous((1024, 1024, 1024), seed=0, device=dev)


def _sampled(got, pts, dev):
    idx = torch.tensor(pts, device=dev)
    if got.dim() == 4:
        return got[:, idx[:, 0], idx[:, 1], idx[:, 2]].double().cpu().numpy().T
    return got[idx[:, 0], idx[:, 1], idx[:, 2]].double().cpu().numpy()


@pytest.mark.parametrize("op", ["mean_r1", "mean_r2", "unsharp_s2", "sobel", "hessian_s1", "niblack_r2"])
def test_filters_full_size_sampled(dev, big_f32, op):
    v = big_f32
    shape = tuple(v.shape)
    print("full-size", op, flush=True)
    if op.startswith("mean"):
        r = int(op[-1])
        got = h.mean(v, r)
    elif op == "unsharp_s2":
        r = oracle.gauss_radius(2.0)
        got = h.unsharp(v, 2.0, 1.0)
    elif op == "sobel":
        r = 1
        got = h.edge(v, "sobel")
    elif op == "hessian_s1":
        r = oracle.gauss_radius(1.0)
        got = h.hessian(v, 1.0)
    else:
        r = 2
        got = h.local_threshold(v, "niblack", radius=2, k=-0.2)
    torch.cuda.synchronize()
    pts = sample_points(shape, 48, seed=len(op))
    gvals = _sampled(got, pts, dev)
    del got
    for p, g in zip(pts, gvals):
        win = window_of(v, p, r)
        c = (r, r, r)
        if op.startswith("mean"):
            want, scale = oracle.mean3d(win, r, method="direct")[c], _mean_scale(win, r)[c]
        elif op == "unsharp_s2":
            want, scale = oracle.unsharp3d(win, 2.0, 1.0)[c], _unsharp_scale(win, 2.0, 1.0)[c]
        elif op == "sobel":
            want, scale = oracle.edge3d(win, "sobel")[c], _edge_scale(win, "sobel")[c]
        elif op == "hessian_s1":
            want = oracle.hessian3d(win, 1.0)[(slice(None),) + c]
            scale = _hess_scale(win, 1.0)[(slice(None),) + c]
        else:
            out, t = oracle.local_threshold3d(win, "niblack", radius=2, k=-0.2, return_t=True)
            if abs(win[c] - t[c]) > _thr_band(win, "niblack", 2, 1.0, -0.2, 128.0, 0.0)[c]:
                assert g == out[c], (p, g, out[c])
            continue
        assert np.all(np.abs(g - want) <= FP32_GAUSS_TOL * scale), (op, p, g, want)


def test_otsu_full_size(dev):
    v = phantoms.porous_u16((1024, 1024, 1024), seed=0, device=dev)
    print("full-size otsu u16", flush=True)
    out, k = h.otsu(v)
    torch.cuda.synchronize()
    vnp = v.cpu().to(torch.int32).numpy()
    assert k == oracle.otsu_threshold(vnp, 65536)
    pts = sample_points(tuple(v.shape), 256, seed=5)
    idx = torch.tensor(pts, device=dev)
    vs = v.to(torch.int32)[idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy()
    os_ = out[idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy()
    np.testing.assert_array_equal(os_, (vs > k).astype(np.uint8))
    assert int(out.sum(dtype=torch.int64)) == int(np.count_nonzero(vnp > k))
