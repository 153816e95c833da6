"""Helpers shared by the GPU parity tests (inputs, oracle windows, bounds)."""
import numpy as np
import torch

import oracle

# unit roundoff of the storage formats (round to nearest even)
U_BF16 = 2.0 ** -8
U_F16 = 2.0 ** -11

FP32_GAUSS_TOL = 1e-5  # |gpu - oracle| <= 1e-5 * G(|v|)


def to_np64(t) -> np.ndarray:
    if isinstance(t, torch.Tensor):
        t = t.detach().cpu()
        if t.dtype in (torch.bfloat16, torch.float16, torch.uint16):
            t = t.to(torch.float32)
        return t.numpy().astype(np.float64)
    return np.asarray(t, dtype=np.float64)


def gauss_scale(v64: np.ndarray, sigma) -> np.ndarray:
    """Condition scale of a positive-weight stencil: G_sigma(|v|)."""
    return oracle.gaussian3d(np.abs(v64), sigma, method="separable")


def assert_gauss_close(got, want, scale, tol, what=""):
    err = np.abs(got - want)
    bad = err > tol * scale
    if bad.any():
        i = np.unravel_index(np.argmax(err / np.maximum(scale, 1e-300)), err.shape)
        raise AssertionError("%s: %d voxels beyond %.1e * scale; worst at %s got %r want %r scale %r"
                             % (what, int(bad.sum()), tol, i, got[i], want[i], scale[i]))


def reflect_window(v: np.ndarray, p, r):
    """(2r+1)^3 neighbourhood of voxel p with half-sample reflection at the
    volume faces; the oracle's output at the window centre equals the
    volume's output at p for any stencil of radius <= r."""
    idx = []
    for a in range(3):
        n = v.shape[a]
        ii = np.arange(p[a] - r, p[a] + r + 1)
        m = np.mod(ii, 2 * n)
        idx.append(np.where(m < n, m, 2 * n - 1 - m))
    return v[np.ix_(idx[0], idx[1], idx[2])]


def reflected_indices(n, c, r):
    ii = np.arange(c - r, c + r + 1)
    m = np.mod(ii, 2 * n)
    return np.where(m < n, m, 2 * n - 1 - m)


def window_of(t: torch.Tensor, p, r) -> np.ndarray:
    """reflect_window of a (device) tensor, gathered on the device."""
    idx = [torch.as_tensor(reflected_indices(t.shape[a], p[a], r), device=t.device) for a in range(3)]
    w = t.index_select(0, idx[0]).index_select(1, idx[1]).index_select(2, idx[2])
    return to_np64(w)


def sample_points(shape, n, seed=0, r=0):
    """Seeded sample voxels: the 8 corners, face centres and random ones."""
    rng = np.random.default_rng(seed)
    pts = set()
    for cz in (0, shape[0] - 1):
        for cy in (0, shape[1] - 1):
            for cx in (0, shape[2] - 1):
                pts.add((cz, cy, cx))
    for a in range(3):
        for side in (0, shape[a] - 1):
            p = [s // 2 for s in shape]
            p[a] = side
            pts.add(tuple(p))
    while len(pts) < n:
        pts.add(tuple(int(rng.integers(0, s)) for s in shape))
    return sorted(pts)


def fp32_gauss_rel_bound(r: int) -> float:
    """Worst-case relative error of an FP32 separable Gaussian of radius r
    against FP64: three passes of 2r+1 products and sums with taps rounded
    to FP32, each step within 2^-24 of its exact value, scaled by G(|x|)."""
    return 3 * (2 * r + 1) * 2.0 ** -24


def near_ties(y64: np.ndarray, r: int, rel: float) -> np.ndarray:
    """Voxels whose box-(2r+1) window (offsets outside the volume skipped)
    has its top two values within rel * max|y|.  With rel twice the error
    bound of the values y, an FP32 and an FP64 argmax can differ only at
    these voxels; everywhere else the routing is unique."""
    from numpy.lib.stride_tricks import sliding_window_view
    p = np.pad(y64, r, mode="constant", constant_values=-np.inf)
    w = sliding_window_view(p, (2 * r + 1,) * 3).reshape(y64.shape + (-1,))
    top2 = -np.partition(-w, 1, axis=-1)[..., :2]
    return (top2[..., 0] - top2[..., 1]) <= rel * np.max(np.abs(y64))
