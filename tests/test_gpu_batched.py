"""Batched persistent launches over uneven crops: bitwise equal to the
per-crop launches (same tile code), gradients of the batched differentiable
workload against the FP64 oracle, and CUDA/HIP-graph replays equal to eager
runs."""
import numpy as np
import pytest
import torch

import oracle
import paper_2511_11890_amd as h
from paper_2511_11890_amd import phantoms
from tests.gpu_util import fp32_gauss_rel_bound, near_ties, to_np64

pytestmark = pytest.mark.gpu


def _crops(dev, n=40, lo=5, hi=90, seed=51):
    parent = phantoms.porous((96, 100, 110), seed=seed).to(dev)
    boxes = phantoms.crop_boxes(n, lo, hi, parent=(96, 100, 110), seed=seed)
    return [parent[z:z + dz, y:y + dy, x:x + dx].contiguous() for (z, y, x), (dz, dy, dx) in boxes]


@pytest.mark.parametrize("sigma", [0.5, 1.0, 1.5, 4.0])
def test_gaussian_batched_equals_per_crop(dev, sigma):
    xs = _crops(dev)
    got = h.gaussian_batched(xs, sigma)
    for x, g in zip(xs, got):
        assert torch.equal(g, h.gaussian(x, sigma))


@pytest.mark.parametrize("op,se,r", [("dilate", "box", 2), ("erode", "ball", 3), ("dilate", "box", 1)])
def test_morph_batched_equals_per_crop(dev, op, se, r):
    xs = _crops(dev, seed=52)
    got = h.morph_batched(xs, op, se, r)
    e, d = h.morph_batched(xs, "erode", se, r), None
    ee = [torch.empty_like(x) for x in xs]
    dd = [torch.empty_like(x) for x in xs]
    h.morph_batched(xs, "erode", se, r, outs=ee, outs2=dd)
    f = h.erode if op == "erode" else h.dilate
    for i, x in enumerate(xs):
        assert torch.equal(got[i], f(x, se, r))
        assert torch.equal(ee[i], h.erode(x, se, r))
        assert torch.equal(dd[i], h.dilate(x, se, r))
    del e, d


def _per_crop_sigma_grad(x, gy):
    _, gs = h.gaussian_backward(x, gy, 1.5, (5, 5, 5), grad_in=False, sigma_sum=True)
    return float(gs[0])


def test_batched_backward_equals_per_crop(dev):
    xs = _crops(dev, n=36, seed=53)
    gds = [phantoms.gaussian_noise(x.shape, seed=54 + i).to(dev) for i, x in enumerate(xs)]
    b = h.GaussDilateBatch(xs, 1.5, "box", 2)
    ds = b.forward()
    gxs, gs = b.backward(gds)
    torch.cuda.synchronize()
    assert gs.shape == (1,)
    tot, mag = 0.0, 0.0
    for x, d, gd, gx in zip(xs, ds, gds, gxs):
        y = h.gaussian(x, 1.5)
        assert torch.equal(d, h.dilate(y, "box", 2))
        gy = h.morph_backward(y, gd, "dilate", "box", 2)
        gi, _ = h.gaussian_backward(x, gy, 1.5, (5, 5, 5), grad_sigma=False)
        assert torch.equal(gx, gi)
        t = _per_crop_sigma_grad(x, gy)
        tot += t
        mag += abs(t)
    # same FP32 products, workgroup partials grouped differently
    assert abs(gs.item() - tot) <= 1e-5 * mag


def _oracle_check(x, c, gx, what):
    """The composite gradient of one crop against the FP64 oracle with the
    near-tie outputs of the dilation masked out of c (where FP32 and FP64
    may route to different maxima); every other voxel within 1e-5 of its
    scale.  Returns (oracle sigma-gradient of the masked loss, the GPU's
    per-crop sigma-gradient of the same masked loss, magnitude)."""
    x64 = to_np64(x)
    y64 = oracle.gaussian3d(x64, 1.5, radius=5, method="separable")
    ties = near_ties(y64, 2, 2 * fp32_gauss_rel_bound(5))
    assert ties.mean() < 5e-3, (what, ties.mean())
    c64 = to_np64(c)
    c64[ties] = 0.0
    L, gxo, gso, _ = oracle.gauss_dilate_loss_grad(x64, c64, 1.5, "box", 2)
    scale = oracle.gaussian3d_transpose(
        np.abs(oracle.morph3d_backward(y64, c64, "dilate", "box", 2)), 1.5, radius=5)
    return ties, gxo, gso, scale


def test_batched_gradient_vs_oracle(dev):
    # L = sum_i sum c_i * dilate_box5(G_sigma x_i), sigma = 1.5 (r = 5); the
    # near-tie outputs are masked out of every c_i before the GPU run too
    xs = _crops(dev, n=5, lo=12, hi=30, seed=55)
    cs = [phantoms.gaussian_noise(x.shape, seed=60 + i).to(dev) for i, x in enumerate(xs)]
    prep = []
    for i, (x, c) in enumerate(zip(xs, cs)):
        ties, gxo, gso, scale = _oracle_check(x, c, None, i)
        c[torch.from_numpy(ties).to(dev)] = 0.0
        prep.append((gxo, gso, scale))
    b = h.GaussDilateBatch(xs, 1.5, "box", 2)
    b.forward()
    gxs, gs = b.backward(cs)
    torch.cuda.synchronize()
    gs_total, gs_mag = 0.0, 0.0
    for gx, (gxo, gso, scale) in zip(gxs, prep):
        err = np.abs(to_np64(gx) - gxo)
        assert np.all(err <= 1e-5 * scale + 1e-7), float(np.max(err - 1e-5 * scale))
        gs_total += gso
        gs_mag += abs(gso)
    assert abs(gs.item() - gs_total) <= 1e-4 * abs(gs_total) + 1e-6 * gs_mag


def _kernel_nodes(graph) -> int:
    """Kernel nodes of a captured graph (hipGraphGetNodes / NodeGetType of the
    HIP runtime torch has loaded)."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so.7")
    g = ctypes.c_void_p(graph.raw_cuda_graph())
    n = ctypes.c_size_t(0)
    assert hip.hipGraphGetNodes(g, None, ctypes.byref(n)) == 0
    nodes = (ctypes.c_void_p * n.value)()
    assert hip.hipGraphGetNodes(g, nodes, ctypes.byref(n)) == 0
    kinds = []
    for i in range(n.value):
        t = ctypes.c_int(-1)
        assert hip.hipGraphNodeGetType(ctypes.c_void_p(nodes[i]), ctypes.byref(t)) == 0
        kinds.append(t.value)
    return sum(1 for k in kinds if k == 0)  # hipGraphNodeTypeKernel


def test_c5_batch_sizes_one_launch_per_kernel(dev):
    """The differentiable batched workload at its own sizes: 64 float32
    crops with seeded extents U[64, 256] per axis, Gaussian sigma 1.5 then
    box-5 dilation.  One training step captures one launch per batched
    kernel (no split of the 64 crops); results equal the per-crop launches;
    the three smallest crops are checked against the FP64 oracle."""
    parent = phantoms.porous((320, 320, 320), seed=57, device=dev)
    boxes = phantoms.crop_boxes(64, 64, 256, parent=(320, 320, 320), seed=57)
    xs = [parent[z:z + dz, y:y + dy, x:x + dx].contiguous() for (z, y, x), (dz, dy, dx) in boxes]
    del parent
    cs = [phantoms.gaussian_noise(x.shape, seed=200 + i, device=dev) for i, x in enumerate(xs)]
    small = sorted(range(len(xs)), key=lambda i: xs[i].numel())[:3]
    prep = {}
    for i in small:
        ties, gxo, gso, scale = _oracle_check(xs[i], cs[i], None, i)
        cs[i][torch.from_numpy(ties).to(dev)] = 0.0
        prep[i] = (gxo, gso, scale)
    b = h.GaussDilateBatch(xs, 1.5, "box", 2)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.forward()
        b.backward(cs)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph(keep_graph=True)
    with torch.cuda.graph(g):
        b.forward()
        b.backward(cs)
    launches = _kernel_nodes(g)
    # forward: Gaussian, dilation with its extremum codes; backward: gather
    # through the codes, Gaussian of the routed gradient, sigma terms, FP64
    # reduction
    assert launches == 6, launches
    for t in b.ds + b.gxs:
        t.zero_()
    g.replay()
    torch.cuda.synchronize()
    tot, mag = 0.0, 0.0
    for i, (x, c) in enumerate(zip(xs, cs)):
        y = h.gaussian(x, 1.5)
        assert torch.equal(b.ds[i], h.dilate(y, "box", 2)), i
        gy = h.morph_backward(y, c, "dilate", "box", 2)
        gi, _ = h.gaussian_backward(x, gy, 1.5, (5, 5, 5), grad_sigma=False)
        assert torch.equal(b.gxs[i], gi), i
        t = _per_crop_sigma_grad(x, gy)
        tot += t
        mag += abs(t)
        if i in prep:
            gxo, gso, scale = prep[i]
            err = np.abs(to_np64(b.gxs[i]) - gxo)
            assert np.all(err <= 1e-5 * scale + 1e-7), (i, float(np.max(err - 1e-5 * scale)))
            assert abs(t - gso) <= 1e-4 * abs(gso) + 1e-6, (i, t, gso)
    assert abs(b.gsigma.item() - tot) <= 1e-5 * mag


@pytest.mark.parametrize("op,se,r", [("dilate", "box", 2), ("erode", "ball", 3), ("erode", "box", 1),
                                     ("dilate", "ball", 2)])
def test_forward_codes_reused_by_backward(dev, op, se, r):
    # harpia_morph3d_forward_batched: the erosion / dilation equals the
    # per-crop call, and the backward through its kept codes equals the
    # backward that recomputes them (and the per-crop subgradient)
    xs = _crops(dev, n=20, seed=58)
    gds = [phantoms.gaussian_noise(x.shape, seed=300 + i).to(dev) for i, x in enumerate(xs)]
    lib = h._lib.load()
    code = {"erode": h._lib.HARPIA_ERODE, "dilate": h._lib.HARPIA_DILATE}[op]
    sc = {"box": 0, "ball": 1}[se]
    outs = [torch.empty_like(x) for x in xs]
    c_fwd = h._lib.crops([(x, o, None) for x, o in zip(xs, outs)])
    ws = torch.empty(int(lib.harpia_batch_workspace_bytes(c_fwd, len(xs))), dtype=torch.uint8, device=dev)
    st = lambda f=0: h._lib.make_exec(stream=torch.cuda.current_stream().cuda_stream, flags=f)  # noqa: E731
    r3 = h._lib.i32_3((r, r, r))
    h._lib.check(lib.harpia_morph3d_forward_batched(c_fwd, len(xs), code, sc, r3, ws.data_ptr(), ws.numel(), st()))
    g_reuse = [torch.empty_like(x) for x in xs]
    h._lib.check(lib.harpia_morph3d_backward_batched(
        h._lib.crops([(None, gi, gd) for gi, gd in zip(g_reuse, gds)]), len(xs), code, sc, r3, ws.data_ptr(),
        ws.numel(), st(h._lib.HARPIA_F_REUSE_CODES)))
    g_new = [torch.empty_like(x) for x in xs]
    h._lib.check(lib.harpia_morph3d_backward_batched(
        h._lib.crops([(x, gi, gd) for x, gi, gd in zip(xs, g_new, gds)]), len(xs), code, sc, r3, ws.data_ptr(),
        ws.numel(), st()))
    torch.cuda.synchronize()
    f = h.erode if op == "erode" else h.dilate
    for x, o, gd, a, b in zip(xs, outs, gds, g_reuse, g_new):
        assert torch.equal(o, f(x, se, r))
        assert torch.equal(a, b)
        assert torch.equal(a, h.morph_backward(x, gd, op, se, r))


def test_graph_replay_equals_eager(dev):
    xs = _crops(dev, n=24, seed=56)
    gds = [phantoms.gaussian_noise(x.shape, seed=70 + i).to(dev) for i, x in enumerate(xs)]
    b = h.GaussDilateBatch(xs, 1.5, "box", 2)
    # eager reference
    b.forward()
    gx_ref, gs_ref = b.backward(gds)
    d_ref = [d.clone() for d in b.ds]
    gx_ref = [g.clone() for g in gx_ref]
    gs_ref = gs_ref.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm-up on the capture stream
        b.forward()
        b.backward(gds)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.forward()
        b.backward(gds)
    for rep in range(3):
        for t in b.ds + b.gxs:
            t.zero_()
        b.gsigma.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for d, r in zip(b.ds, d_ref):
            assert torch.equal(d, r), rep
        for gx, r in zip(b.gxs, gx_ref):
            assert torch.equal(gx, r), rep
        assert torch.equal(b.gsigma, gs_ref), rep
        h.gaussian(xs[0], 2.0)  # unrelated eager work between replays
