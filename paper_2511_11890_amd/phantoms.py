"""Seeded synthetic tomography-like volumes (inputs only).

This module generates inputs for the tests, the smoke check and the
benchmark.  It holds none of the filters' arithmetic: no reflect-boundary
stencil, no erosion or dilation, no Gaussian tap.  The smoothing used to give
the porous phantom a correlation length is a periodic three-pass box blur,
which is a different operator from the filters under test.

The paper evaluates on a real synchrotron tomogram (Section IV-A) that is not
available; these phantoms stand in for it with the structure of the paper's
domain (two-phase porous media, blob-like features, additive noise).

Recipes
  blobs(n)        : sum of 40 isotropic Gaussian blobs (centres U[0, n)^3,
                    width U[4, 12] voxels, amplitude U[0.2, 1]) evaluated in
                    FP64, plus N(0, 0.05) noise, cast to float32.
  porous(shape)   : N(0, 1) noise, blurred by periodic box filters of widths
                    7, 7, 3 along every axis (effective sigma 2.94 voxels),
                    thresholded at its 40th percentile into phases 0.3 / 0.7,
                    plus N(0, 0.05) noise; float32.
  porous_u16      : round(clip(v, 0, 1) * 65535) of porous().
  porous_16bit    : clip(v, 0, 1) rounded to bfloat16 / float16 (RNE).
  crops           : seeded uneven crop sizes in [lo, hi] per axis and seeded
                    offsets into a parent volume.
"""
from __future__ import annotations

import numpy as np
import torch

# Effective sigma of three box passes of widths w: sqrt(sum (w^2 - 1) / 12).
BOX_WIDTHS = (7, 7, 3)


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=[seed, stream]))


def _torch_gen(seed: int, stream: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed((int(seed) * 1000003 + int(stream)) & 0x7FFFFFFFFFFFFFFF)
    return g


def blobs(n: int = 128, n_blobs: int = 40, noise: float = 0.05,
          seed: int = 0, shape=None) -> np.ndarray:
    """Sum of isotropic Gaussian blobs plus white noise (float32, [n, n, n],
    or `shape` with centres uniform over each extent)."""
    shape = (n, n, n) if shape is None else tuple(int(s) for s in shape)
    rng = _rng(seed, 1)
    centres = rng.uniform(0.0, 1.0, size=(n_blobs, 3)) * np.array(shape, dtype=np.float64)
    widths = rng.uniform(4.0, 12.0, size=n_blobs)
    amps = rng.uniform(0.2, 1.0, size=n_blobs)
    axes = [np.arange(s, dtype=np.float64) for s in shape]
    v = np.zeros(shape, dtype=np.float64)
    for (cz, cy, cx), s, a in zip(centres, widths, amps):
        ez = np.exp(-((axes[0] - cz) ** 2) / (2 * s * s))
        ey = np.exp(-((axes[1] - cy) ** 2) / (2 * s * s))
        ex = np.exp(-((axes[2] - cx) ** 2) / (2 * s * s))
        v += a * ez[:, None, None] * ey[None, :, None] * ex[None, None, :]
    v += rng.normal(0.0, noise, size=v.shape)
    return v.astype(np.float32)


def _box_blur_periodic(t: torch.Tensor, width: int, dim: int) -> torch.Tensor:
    h = width // 2
    acc = t.clone()
    for k in range(1, h + 1):
        acc += torch.roll(t, k, dims=dim)
        acc += torch.roll(t, -k, dims=dim)
    return acc / float(width)


def porous(shape=(128, 128, 128), noise: float = 0.05, seed: int = 0,
           device="cpu", pct: float = 40.0) -> torch.Tensor:
    """Two-phase porous-medium phantom, float32 torch tensor on `device`."""
    shape = tuple(int(s) for s in shape)
    g = _torch_gen(seed, 2, device)
    s = torch.randn(shape, generator=g, device=device, dtype=torch.float32)
    for dim in range(3):
        for w in BOX_WIDTHS:
            s = _box_blur_periodic(s, w, dim)
    flat = s.reshape(-1)
    if flat.numel() <= (1 << 24):
        sample = flat
    else:
        gi = _torch_gen(seed, 3, device)
        idx = torch.randint(0, flat.numel(), (1 << 24,), generator=gi, device=device)
        sample = flat[idx]
    k = max(1, int(round(pct / 100.0 * sample.numel())))
    t = torch.kthvalue(sample.float().cpu(), k).values.item()
    v = torch.where(s < t, torch.tensor(0.3, device=device), torch.tensor(0.7, device=device))
    del s
    gn = _torch_gen(seed, 4, device)
    v = v + noise * torch.randn(shape, generator=gn, device=device, dtype=torch.float32)
    return v.to(torch.float32)


def porous_u16(shape=(128, 128, 128), seed: int = 0, device="cpu") -> torch.Tensor:
    """porous() scaled to uint16: round(clip(v, 0, 1) * 65535)."""
    v = porous(shape, seed=seed, device=device)
    q = torch.round(torch.clamp(v, 0.0, 1.0) * 65535.0).to(torch.int32)
    return q.to(torch.uint16)


def porous_16bit(shape=(128, 128, 128), dtype=torch.bfloat16, seed: int = 0,
                 device="cpu"):
    """Return (unquantised float32 values in [0, 1], the same rounded RNE to
    `dtype`)."""
    v = torch.clamp(porous(shape, seed=seed, device=device), 0.0, 1.0)
    return v, v.to(dtype)


def crop_boxes(n: int = 64, lo: int = 64, hi: int = 256, parent=(1024, 1024, 1024),
               seed: int = 0):
    """Seeded uneven crops: list of ((z0, y0, x0), (dz, dy, dx)) inside `parent`."""
    rng = _rng(seed, 5)
    sizes = rng.integers(lo, hi, size=(n, 3), endpoint=True)
    out = []
    for s in sizes:
        origin = tuple(int(rng.integers(0, parent[a] - s[a], endpoint=True)) for a in range(3))
        out.append((origin, tuple(int(t) for t in s)))
    return out


def gaussian_noise(shape, seed: int = 0, stream: int = 6, device="cpu") -> torch.Tensor:
    """Seeded N(0, 1) float32 volume (e.g. the upstream weights c of a loss)."""
    g = _torch_gen(seed, stream, device)
    return torch.randn(tuple(int(s) for s in shape), generator=g, device=device,
                       dtype=torch.float32)
