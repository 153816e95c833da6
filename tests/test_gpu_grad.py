"""GPU parity of the adjoint kernels (the differentiation extension) against
the FP64 oracle: Gaussian input gradient (the oracle's literal transpose),
sigma-gradient (the oracle's d/d sigma convolution), morphology subgradient
(the oracle's first-extremum routing), and the composite loss
L = sum c * dilate_box5(G_sigma x) of the batched workload."""
import numpy as np
import pytest
import torch

import oracle
import paper_2511_11890_amd as h
from paper_2511_11890_amd import phantoms
from tests.gpu_util import FP32_GAUSS_TOL, fp32_gauss_rel_bound, gauss_scale, near_ties, to_np64

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape,sigma", [((37, 45, 150), 1.5), ((30, 40, 100), 2.0), ((20, 33, 70), 4.0),
                                         ((3, 5, 7), 2.0), ((25, 30, 80), (1.0, 2.0, 1.5))])
def test_gaussian_input_gradient_is_literal_transpose(dev, shape, sigma):
    g = phantoms.gaussian_noise(shape, seed=31).numpy()
    r = tuple(oracle.gauss_radius(s) for s in (sigma if isinstance(sigma, tuple) else (sigma,) * 3))
    gi, _ = h.gaussian_backward(None, torch.from_numpy(g).to(dev), sigma, r, grad_sigma=False)
    torch.cuda.synchronize()
    g64 = g.astype(np.float64)
    want = oracle.gaussian3d_transpose(g64, sigma, radius=r)
    scale = oracle.gaussian3d_transpose(np.abs(g64), sigma, radius=r)
    got = to_np64(gi)
    assert np.all(np.abs(got - want) <= FP32_GAUSS_TOL * scale)


@pytest.mark.parametrize("shape,sigma", [((37, 45, 150), 1.5), ((30, 40, 100), (1.2, 1.6, 2.1)),
                                         ((24, 30, 90), 4.0), ((2, 3, 70), 1.0)])
@pytest.mark.parametrize("xdtype", [torch.float32, torch.uint16])
def test_gaussian_sigma_gradient(dev, shape, sigma, xdtype):
    x = phantoms.porous(shape, seed=32)
    if xdtype == torch.uint16:
        x = phantoms.porous_u16(shape, seed=32)
    g = phantoms.gaussian_noise(shape, seed=33)
    s3 = sigma if isinstance(sigma, tuple) else (sigma,) * 3
    r = tuple(oracle.gauss_radius(s) for s in s3)
    _, gs = h.gaussian_backward(x.to(dev), g.to(dev), s3, r, grad_in=False)
    torch.cuda.synchronize()
    x64, g64 = to_np64(x), to_np64(g)
    for a in range(3):
        d = oracle.gaussian3d_dsigma_axis(x64, s3, a, radius=r)
        want = float(np.sum(g64 * d))
        mag = float(np.sum(np.abs(g64 * d)))
        # FP32 products and per-block sums: error well below 1e-5 of the
        # sum of magnitudes
        assert abs(gs[a].item() - want) <= 1e-5 * mag, (a, gs[a].item(), want, mag)


def test_sigma_gradient_host_pointer_and_deterministic(dev):
    shape = (40, 50, 130)
    x = phantoms.porous(shape, seed=34).to(dev)
    g = phantoms.gaussian_noise(shape, seed=35).to(dev)
    _, a = h.gaussian_backward(x, g, 2.0, (6, 6, 6), grad_in=False)
    _, b = h.gaussian_backward(x, g, 2.0, (6, 6, 6), grad_in=False)
    assert torch.equal(a, b)
    out = np.zeros(3)
    lib = h._lib.load()
    h._lib.check(lib.harpia_gaussian3d_backward(
        x.data_ptr(), h._lib.HARPIA_F32, g.data_ptr(), None, h._lib.i64_3(shape), h._lib.f64_3((2.0,) * 3),
        h._lib.i32_3((6, 6, 6)), out.ctypes.data, h._lib.make_exec(stream=torch.cuda.current_stream().cuda_stream)))
    np.testing.assert_array_equal(out, a.cpu().numpy())


@pytest.mark.parametrize("sigma,r", [(2.0, (6, 6, 6)), ((1.0, 1.5, 2.0), (3, 5, 6))])
def test_sigma_gradient_sum_flag(dev, sigma, r):
    # HARPIA_F_SIGMA_SUM: one FP64 value, the sum of the three axis terms,
    # into a device pointer and (through the raw C ABI) a host pointer; the
    # unfused path (unequal radii) sums its per-axis reductions
    shape = (22, 37, 90)
    x = phantoms.porous(shape, seed=45).to(dev)
    g = phantoms.gaussian_noise(shape, seed=46).to(dev)
    _, g3 = h.gaussian_backward(x, g, sigma, r, grad_in=False)
    _, g1 = h.gaussian_backward(x, g, sigma, r, grad_in=False, sigma_sum=True)
    torch.cuda.synchronize()
    assert g1.shape == (1,)
    want = float(g3.sum())
    assert abs(float(g1[0]) - want) <= 1e-12 * float(g3.abs().sum())
    out = np.full(3, 7.0)
    lib = h._lib.load()
    h._lib.check(lib.harpia_gaussian3d_backward(
        x.data_ptr(), h._lib.HARPIA_F32, g.data_ptr(), None, h._lib.i64_3(shape),
        h._lib.f64_3(h._triple(sigma, float)), h._lib.i32_3(r), out.ctypes.data,
        h._lib.make_exec(stream=torch.cuda.current_stream().cuda_stream, flags=h._lib.HARPIA_F_SIGMA_SUM)))
    assert out[0] == float(g1[0])
    assert out[1] == 7.0 and out[2] == 7.0  # one value written


@pytest.mark.parametrize("op", ["erode", "dilate"])
@pytest.mark.parametrize("se,r", [("box", 1), ("box", 2), ("ball", 2), ("ball", 3), ("box", (1, 2, 0)),
                                  ("box", (3, 1, 4)), ("box", 8), ("ball", 4)])
def test_morph_gradient_ties_exact(dev, op, se, r):
    # integer data with many ties and integer upstream gradients: the sums
    # are exact in FP32, so the tie rule must match the oracle bit for bit
    shape = (13, 21, 70)
    rng = np.random.default_rng(36)
    v = rng.integers(0, 3, size=shape).astype(np.float32)
    g = rng.integers(-3, 4, size=shape).astype(np.float32)
    gi = h.morph_backward(torch.from_numpy(v).to(dev), torch.from_numpy(g).to(dev), op, se, r)
    torch.cuda.synchronize()
    want = oracle.morph3d_backward(v.astype(np.float64), g.astype(np.float64), op, se, r)
    np.testing.assert_array_equal(to_np64(gi), want)


def test_morph_gradient_limits(dev):
    v = torch.zeros((8, 9, 10), device=dev)
    with pytest.raises(h.HarpiaError):
        h.morph_backward(v, v, "dilate", "ball", 5)
    with pytest.raises(h.HarpiaError):
        h.morph_backward(v, v, "dilate", "box", 9)


def test_morph_gradient_large_ragged(dev):
    # several tiles in x and y, several z ranges, ragged tails on every axis
    shape = (150, 77, 203)
    rng = np.random.default_rng(41)
    v = rng.integers(0, 5, size=shape).astype(np.float32)
    g = rng.integers(-3, 4, size=shape).astype(np.float32)
    for op in ("erode", "dilate"):
        gi = h.morph_backward(torch.from_numpy(v).to(dev), torch.from_numpy(g).to(dev), op, "box", (2, 3, 1))
        torch.cuda.synchronize()
        want = oracle.morph3d_backward(v.astype(np.float64), g.astype(np.float64), op, "box", (2, 3, 1))
        np.testing.assert_array_equal(to_np64(gi), want)


@pytest.mark.parametrize("dtype", [torch.float32, torch.uint16, torch.bfloat16, torch.uint8, torch.float16])
def test_morph_gradient_dtypes(dev, dtype):
    shape = (17, 29, 90)
    v = phantoms.porous(shape, seed=37)
    if dtype == torch.uint16:
        v = phantoms.porous_u16(shape, seed=37)
    elif dtype == torch.uint8:
        v = (phantoms.porous_u16(shape, seed=37).to(torch.int32) >> 8).to(torch.uint8)
    elif dtype in (torch.bfloat16, torch.float16):
        v = torch.clamp(v, 0, 1).to(dtype)
    g = phantoms.gaussian_noise(shape, seed=38)
    gi = h.morph_backward(v.to(dev), g.to(dev), "dilate", "box", 2)
    torch.cuda.synchronize()
    want = oracle.morph3d_backward(to_np64(v), to_np64(g), "dilate", "box", 2)
    mag = oracle.morph3d_backward(to_np64(v), np.abs(to_np64(g)), "dilate", "box", 2)
    assert np.all(np.abs(to_np64(gi) - want) <= 125 * 2.0 ** -24 * mag)


def test_composite_loss_gradient_vs_oracle(dev):
    """L = sum c * dilate_box5(G_sigma x), sigma = 1.5 (r = 5): input and sigma
    gradients from GaussDilateFn against the FP64 oracle.  Outputs whose
    dilation window has a near-tie (top-two gap within twice the FP32
    Gaussian's error bound, where FP32 and FP64 may pick different maxima)
    are masked out of c.  Their share is a property of the input (a smooth
    field has near-equal neighbours around each local maximum, and a maximum
    is the window maximum of up to 125 outputs): 0.27% here; the bound only
    keeps the mask from swallowing the check."""
    shape = (30, 41, 96)
    x = phantoms.porous(shape, seed=39)
    c = phantoms.gaussian_noise(shape, seed=40)
    y64 = oracle.gaussian3d(to_np64(x), 1.5, method="separable")
    ties = near_ties(y64, 2, 2 * fp32_gauss_rel_bound(5))
    assert ties.mean() < 5e-3
    c[torch.from_numpy(ties)] = 0.0
    xd = x.to(dev).requires_grad_(True)
    sig = torch.tensor(1.5, dtype=torch.float64, requires_grad=True)
    d = h.GaussDilateFn.apply(xd, sig, "box", 2)
    loss = (c.to(dev) * d).sum()
    loss.backward()
    torch.cuda.synchronize()
    L, gx, gs, _ = oracle.gauss_dilate_loss_grad(to_np64(x), to_np64(c), 1.5, "box", 2)
    assert abs(loss.item() - L) <= 1e-5 * np.sum(np.abs(to_np64(c)) * np.abs(y64).max())
    gxs = oracle.gaussian3d_transpose(np.abs(oracle.morph3d_backward(y64, to_np64(c), "dilate", "box", 2)), 1.5,
                                      radius=5)
    assert np.all(np.abs(to_np64(xd.grad) - gx) <= 1e-5 * gxs + 1e-7)
    assert abs(sig.grad.item() - gs) <= 1e-4 * abs(gs) + 1e-6


def test_composite_sigma_gradient_vs_gpu_finite_difference(dev):
    # central difference of the GPU forward, h = 1e-3, radius held at 5
    shape = (24, 33, 80)
    x = phantoms.porous(shape, seed=41).to(dev)
    c = phantoms.gaussian_noise(shape, seed=42).to(dev)
    sig = torch.tensor(1.5, dtype=torch.float64, requires_grad=True)
    (c * h.GaussDilateFn.apply(x, sig, "box", 2)).sum().backward()

    def L(s):
        y = h.gaussian(x, s, truncate=5.0 / s)  # r = int(5.0 + 0.5) = 5, held fixed
        return float((c.double() * h.dilate(y, "box", 2).double()).sum())

    hh = 1e-3
    fd = (L(1.5 + hh) - L(1.5 - hh)) / (2 * hh)
    assert abs(sig.grad.item() - fd) <= 2e-2 * abs(fd) + 5e-2


def test_gaussian_fn_autograd(dev):
    shape = (20, 30, 70)
    x = phantoms.porous(shape, seed=43).to(dev).requires_grad_(True)
    g = phantoms.gaussian_noise(shape, seed=44).to(dev)
    sig = torch.tensor([1.0, 1.5, 2.0], dtype=torch.float64, requires_grad=True)
    (g * h.GaussianFn.apply(x, sig)).sum().backward()
    r = (3, 5, 6)
    gi, gs = h.gaussian_backward(x.detach(), g, (1.0, 1.5, 2.0), r)
    assert torch.equal(x.grad, gi)
    assert torch.equal(sig.grad, gs.cpu())
