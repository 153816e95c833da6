"""Pins of the FP64 oracle against things other than itself.

The paper names Gaussian smoothing, erosion, dilation and opening (Section
III-C) but prints no outputs, so each oracle function is pinned by
  - a library special case (scipy.ndimage, only called),
  - pure-Python brute force on tiny volumes (padding by numpy, not by the
    oracle's reflect),
  - closed forms and hand-worked fixtures under tests/golden/,
  - invariants fixed by the mathematics (constant volume, impulse, linearity,
    adjointness, symmetry of the reflect operator, order, duality,
    idempotence, separability, finite differences).
Each is chosen so that a plausible slip (dropped term, wrong sign or index,
transposed operand, off-by-one in the reflect) fails at least one test.
"""
import itertools
import math
import os

import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng(seed=0):
    return np.random.default_rng(seed)


def _load_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([float(t) for t in line.split()])
    return np.array(rows)


def _ball(r):
    d = np.arange(-r, r + 1)
    return (d[:, None, None] ** 2 + d[None, :, None] ** 2 + d[None, None, :] ** 2) <= r * r


def _box(r):
    rz, ry, rx = (r, r, r) if np.ndim(r) == 0 else r
    return np.ones((2 * rz + 1, 2 * ry + 1, 2 * rx + 1), dtype=bool)


# ------------------------------------------------------------------ reflect

def test_reflect_golden():
    g = _load_golden("reflect_n4.txt")
    for i, want in g:
        assert oracle.reflect(int(i), 4) == int(want)


@pytest.mark.parametrize("n", [1, 2, 3, 7])
def test_reflect_matches_numpy_symmetric_pad(n):
    pad = 3 * n + 5
    line = np.pad(np.arange(n), pad, mode="symmetric")
    for j, want in enumerate(line):
        assert oracle.reflect(j - pad, n) == want


# ------------------------------------------------------------------ taps

def test_taps_golden_sigma1():
    g = _load_golden("taps_sigma1.txt")
    assert oracle.gauss_radius(1.0, 3.0) == 3
    w = oracle.gauss_taps(1.0, 3)
    for k, want in g:
        assert w[3 + int(k)] == pytest.approx(want, rel=1e-15, abs=0)
        assert w[3 - int(k)] == pytest.approx(want, rel=1e-15, abs=0)


@pytest.mark.parametrize("sigma,r", [(1.0, 3), (1.5, 5), (2.0, 6), (3.0, 9), (4.0, 12)])
def test_radius_rule(sigma, r):
    assert oracle.gauss_radius(sigma, 3.0) == r


def test_radius_jump_at_1p5():
    # int(3 sigma + 0.5) drops from 5 to 4 just below sigma = 1.5
    assert oracle.gauss_radius(1.5, 3.0) == 5
    assert oracle.gauss_radius(1.499, 3.0) == 4


@pytest.mark.parametrize("sigma", [0.5, 1.0, 1.5, 2.0, 4.0])
def test_taps_equal_scipy_impulse_response(sigma):
    r = oracle.gauss_radius(sigma, 3.0)
    n = 2 * r + 1 + 10
    d = np.zeros(n)
    d[n // 2] = 1.0
    resp = ndi.gaussian_filter1d(d, sigma, mode="reflect", truncate=3.0)
    w = oracle.gauss_taps(sigma, r)
    np.testing.assert_allclose(resp[n // 2 - r:n // 2 + r + 1], w, rtol=1e-14, atol=1e-17)


@pytest.mark.parametrize("sigma", [0.7, 1.5, 2.0, 4.0])
def test_dtaps_match_finite_difference(sigma):
    r = oracle.gauss_radius(sigma, 3.0)
    h = 1e-5
    fd = (oracle.gauss_taps(sigma + h, r) - oracle.gauss_taps(sigma - h, r)) / (2 * h)
    np.testing.assert_allclose(oracle.gauss_dtaps(sigma, r), fd, rtol=1e-7, atol=1e-11)
    # normalisation is preserved to first order: the derivative taps sum to 0
    assert abs(oracle.gauss_dtaps(sigma, r).sum()) < 1e-15


# ------------------------------------------------------------------ Gaussian

@pytest.mark.parametrize("shape", [(6, 7, 8), (3, 4, 5), (1, 1, 9), (10, 1, 3)])
@pytest.mark.parametrize("sigma", [1.0, 2.0, (0.8, 1.5, 2.5)])
def test_gaussian_direct_equals_scipy(shape, sigma):
    v = _rng(1).standard_normal(shape)
    want = ndi.gaussian_filter(v, sigma, mode="reflect", truncate=3.0)
    got = oracle.gaussian3d(v, sigma, method="direct")
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("sigma", [1.0, 1.5, 2.0, 4.0])
def test_gaussian_separable_equals_direct(sigma):
    v = _rng(2).standard_normal((14, 15, 16))
    a = oracle.gaussian3d(v, sigma, method="direct")
    b = oracle.gaussian3d(v, sigma, method="separable")
    np.testing.assert_allclose(b, a, rtol=1e-13, atol=1e-14)


def _brute_gauss(v, sigma, truncate=3.0):
    """Pure-Python definition: pad by numpy 'symmetric' (repeated for large r)
    and sum w_a w_b w_c over the padded neighbourhood."""
    r = int(truncate * sigma + 0.5)
    e = [math.exp(-(k * k) / (2 * sigma * sigma)) for k in range(-r, r + 1)]
    s = sum(e)
    w = [t / s for t in e]
    p = np.pad(v, r, mode="symmetric")
    nz, ny, nx = v.shape
    out = np.zeros_like(v)
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        acc = 0.0
        for a in range(2 * r + 1):
            for b in range(2 * r + 1):
                for c in range(2 * r + 1):
                    acc += w[a] * w[b] * w[c] * p[z + a, y + b, x + c]
        out[z, y, x] = acc
    return out


@pytest.mark.parametrize("shape,sigma", [((2, 3, 4), 1.0), ((3, 2, 2), 2.0), ((1, 2, 3), 4.0)])
def test_gaussian_brute_force_tiny(shape, sigma):
    # radii 3, 6, 12 exceed the sizes: exercises repeated reflection
    v = _rng(3).standard_normal(shape)
    np.testing.assert_allclose(oracle.gaussian3d(v, sigma), _brute_gauss(v, sigma),
                               rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("sigma", [1.0, 2.0, 4.0])
def test_gaussian_constant_volume(sigma):
    # rounding bound of a sum of N positive terms: N * 2^-53 relative
    v = np.full((5, 9, 13), 0.731)
    r = oracle.gauss_radius(sigma)
    for method, terms in (("direct", (2 * r + 1) ** 3), ("separable", 3 * (2 * r + 1))):
        got = oracle.gaussian3d(v, sigma, method=method)
        assert np.max(np.abs(got - 0.731)) <= 2 * terms * 2.0 ** -53 * 0.731


@pytest.mark.parametrize("sigma", [1.0, 1.5, 2.0, 4.0])
def test_gaussian_interior_impulse_is_outer_product(sigma):
    r = oracle.gauss_radius(sigma)
    n = 2 * r + 5
    v = np.zeros((n, n, n))
    c = n // 2
    v[c, c, c] = 1.0
    got = oracle.gaussian3d(v, sigma, method="separable")
    e = np.array([math.exp(-(k * k) / (2 * sigma * sigma)) for k in range(-r, r + 1)])
    w = e / e.sum()
    want = np.zeros_like(v)
    want[c - r:c + r + 1, c - r:c + r + 1, c - r:c + r + 1] = w[:, None, None] * w[None, :, None] * w[None, None, :]
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-17)


def test_gaussian_face_impulse_is_folded_kernel():
    # impulse on the x = 0 face: the reflected taps fold onto the face voxels
    sigma, r = 1.0, 3
    v = np.zeros((1, 1, 8))
    v[0, 0, 0] = 1.0
    got = oracle.gaussian3d(v, (1e-9, 1e-9, sigma))[0, 0]  # r = 0 on z and y
    w = oracle.gauss_taps(sigma, r)
    want = np.zeros(8)
    for x in range(8):
        for k in range(-r, r + 1):
            src = x + k
            src = -src - 1 if src < 0 else src
            if src == 0:
                want[x] += w[k + r]
    np.testing.assert_allclose(got, want, rtol=1e-14)


def test_gaussian_linearity():
    rng = _rng(4)
    a, b = rng.standard_normal((2, 9, 10, 11))
    lhs = oracle.gaussian3d(2.5 * a - 0.75 * b, 1.5)
    rhs = 2.5 * oracle.gaussian3d(a, 1.5) - 0.75 * oracle.gaussian3d(b, 1.5)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_gaussian_commutes_with_flip(axis):
    v = _rng(5).standard_normal((7, 8, 9))
    a = np.flip(oracle.gaussian3d(v, 2.0), axis)
    b = oracle.gaussian3d(np.flip(v, axis), 2.0)
    np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-14)


# --------------------------------------------------------- adjoint / symmetry

def _dense_matrix_1d(fn, n):
    m = np.zeros((n, n))
    for j in range(n):
        e = np.zeros((1, 1, n))
        e[0, 0, j] = 1.0
        m[:, j] = fn(e)[0, 0]
    return m


@pytest.mark.parametrize("n,sigma", [(1, 1.0), (4, 2.0), (7, 1.0), (20, 4.0), (5, 4.0)])
def test_transpose_is_literal_adjoint_and_symmetric(n, sigma):
    s = (1e-9, 1e-9, sigma)
    A = _dense_matrix_1d(lambda e: oracle.gaussian3d(e, s, method="separable"), n)
    At = _dense_matrix_1d(lambda e: oracle.gaussian3d_transpose(e, s), n)
    np.testing.assert_allclose(At, A.T, rtol=1e-14, atol=1e-16)
    # half-sample reflect makes the 1D operator symmetric, faces included
    np.testing.assert_allclose(A, A.T, rtol=1e-13, atol=1e-16)
    # unit row sums; with symmetry the columns sum to 1 too
    np.testing.assert_allclose(A.sum(axis=1), 1.0, rtol=1e-14)


def test_adjointness_3d():
    rng = _rng(6)
    x, y = rng.standard_normal((2, 6, 9, 5))
    for sigma in (1.0, 2.0, (1.0, 4.0, 1.5)):
        gx = oracle.gaussian3d(x, sigma, method="separable")
        gty = oracle.gaussian3d_transpose(y, sigma)
        lhs, rhs = float(np.sum(gx * y)), float(np.sum(x * gty))
        assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + 1)
        np.testing.assert_allclose(gty, oracle.gaussian3d(y, sigma, method="separable"),
                                   rtol=1e-12, atol=1e-14)


def test_mirror_boundary_would_not_be_symmetric():
    # guard on the reading: with whole-sample mirror the transpose differs,
    # so the symmetry above genuinely depends on the half-sample reflect
    n, sigma = 6, 1.0
    w = oracle.gauss_taps(sigma, 3)
    A = np.zeros((n, n))
    for i in range(n):
        for k in range(-3, 4):
            j = i + k
            j = -j if j < 0 else (2 * n - 2 - j if j >= n else j)
            A[i, j] += w[k + 3]
    assert np.max(np.abs(A - A.T)) > 1e-3


# ------------------------------------------------------------ sigma gradient

@pytest.mark.parametrize("sigma", [1.0, 1.5, 2.0])
def test_dsigma_matches_finite_difference(sigma):
    v = _rng(7).standard_normal((8, 9, 10))
    r = oracle.gauss_radius(sigma)

    def central(h):
        return (oracle.gaussian3d(v, sigma + h, radius=r, method="separable")
                - oracle.gaussian3d(v, sigma - h, radius=r, method="separable")) / (2 * h)

    fd = (4 * central(5e-4) - central(1e-3)) / 3  # Richardson: O(h^4)
    np.testing.assert_allclose(oracle.gaussian3d_dsigma(v, sigma), fd, rtol=1e-7, atol=1e-10)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_dsigma_axis_matches_finite_difference(axis):
    v = _rng(8).standard_normal((7, 8, 9))
    s = [1.2, 1.6, 2.1]
    r = [oracle.gauss_radius(t) for t in s]

    def central(h):
        sp, sm = list(s), list(s)
        sp[axis] += h
        sm[axis] -= h
        return (oracle.gaussian3d(v, sp, radius=r, method="separable")
                - oracle.gaussian3d(v, sm, radius=r, method="separable")) / (2 * h)

    fd = (4 * central(5e-4) - central(1e-3)) / 3
    np.testing.assert_allclose(oracle.gaussian3d_dsigma_axis(v, s, axis, radius=r), fd,
                               rtol=1e-7, atol=1e-10)


# ------------------------------------------------------------------ morphology

def test_morph_golden_line():
    g = _load_golden("morph_line5.txt")
    v = g[:, 1].reshape(1, 1, 5)
    for se, rad in (("box", (0, 0, 1)), ("ball", 1)):
        np.testing.assert_array_equal(oracle.erode3d(v, se, rad)[0, 0], g[:, 2])
        np.testing.assert_array_equal(oracle.dilate3d(v, se, rad)[0, 0], g[:, 3])


@pytest.mark.parametrize("se,r", [("box", 1), ("box", 2), ("box", (1, 2, 3)), ("ball", 1),
                                  ("ball", 2), ("ball", 3)])
@pytest.mark.parametrize("mode", ["reflect", "nearest"])
def test_morph_equals_scipy(se, r, mode):
    v = _rng(9).standard_normal((6, 7, 8))
    fp = _box(r) if se == "box" else _ball(r)
    np.testing.assert_array_equal(oracle.erode3d(v, se, r), ndi.grey_erosion(v, footprint=fp, mode=mode))
    np.testing.assert_array_equal(oracle.dilate3d(v, se, r), ndi.grey_dilation(v, footprint=fp, mode=mode))


@pytest.mark.parametrize("r,count", [(1, 7), (2, 33), (3, 123)])
def test_ball_voxel_counts(r, count):
    # the ball's size equals the number of voxels an impulse dilates into
    n = 2 * r + 3
    v = np.zeros((n, n, n))
    v[n // 2, n // 2, n // 2] = 1.0
    assert int(oracle.dilate3d(v, "ball", r).sum()) == count


def _brute_morph(v, op, offsets):
    nz, ny, nx = v.shape
    out = np.empty_like(v)
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        vals = [v[z + a, y + b, x + c] for a, b, c in offsets
                if 0 <= z + a < nz and 0 <= y + b < ny and 0 <= x + c < nx]
        out[z, y, x] = min(vals) if op == "erode" else max(vals)
    return out


@pytest.mark.parametrize("se,r", [("box", 1), ("ball", 2), ("box", (0, 1, 2))])
def test_morph_brute_force_tiny(se, r):
    v = _rng(10).integers(0, 7, size=(4, 3, 5)).astype(float)
    rr = (r, r, r) if np.ndim(r) == 0 else r
    offs = [(a, b, c) for a in range(-rr[0], rr[0] + 1) for b in range(-rr[1], rr[1] + 1)
            for c in range(-rr[2], rr[2] + 1)
            if se == "box" or a * a + b * b + c * c <= rr[0] ** 2]
    for op in ("erode", "dilate"):
        np.testing.assert_array_equal(oracle.morph3d(v, op, se, r), _brute_morph(v, op, offs))


def test_morph_order_duality_separability():
    rng = _rng(11)
    f = rng.integers(0, 65536, size=(9, 10, 11)).astype(float)
    for se, r in (("box", 2), ("ball", 3)):
        e, d = oracle.erode3d(f, se, r), oracle.dilate3d(f, se, r)
        assert np.all(e <= f) and np.all(f <= d)
        np.testing.assert_array_equal(d, 65535 - oracle.erode3d(65535 - f, se, r))
        np.testing.assert_array_equal(d, -oracle.erode3d(-f, se, r))
    # box erosion = erosion along x, then y, then z
    sep = oracle.erode3d(oracle.erode3d(oracle.erode3d(f, "box", (0, 0, 2)), "box", (0, 1, 0)),
                         "box", (3, 0, 0))
    np.testing.assert_array_equal(sep, oracle.erode3d(f, "box", (3, 1, 2)))


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_morph_commutes_with_flip(axis):
    f = _rng(12).standard_normal((5, 6, 7))
    for op in ("erode", "dilate"):
        a = np.flip(oracle.morph3d(f, op, "ball", 2), axis)
        b = oracle.morph3d(np.flip(f, axis), op, "ball", 2)
        np.testing.assert_array_equal(a, b)


def test_opening_closing_properties():
    b = (_rng(13).random((12, 13, 14)) > 0.45).astype(float)
    for se, r in (("box", 1), ("ball", 2)):
        o = oracle.opening3d(b, se, r)
        assert np.all(o <= b)                                  # anti-extensive
        np.testing.assert_array_equal(oracle.opening3d(o, se, r), o)  # idempotent
        c = oracle.closing3d(b, se, r)
        assert np.all(c >= b)                                  # extensive
        np.testing.assert_array_equal(oracle.closing3d(c, se, r), c)


@pytest.mark.parametrize("se,r", [("box", 1), ("ball", 2)])
def test_binary_equals_scipy_binary(se, r):
    b = _rng(14).random((9, 10, 11)) > 0.4
    fp = _box(r) if se == "box" else _ball(r)
    # outside the volume is neutral: 1 for erosion (AND), 0 for dilation (OR)
    want_e = ndi.binary_erosion(b, structure=fp, border_value=1)
    want_d = ndi.binary_dilation(b, structure=fp, border_value=0)
    np.testing.assert_array_equal(oracle.erode3d(b.astype(float), se, r), want_e.astype(float))
    np.testing.assert_array_equal(oracle.dilate3d(b.astype(float), se, r), want_d.astype(float))
    np.testing.assert_array_equal(oracle.opening3d(b.astype(float), se, r),
                                  ndi.binary_dilation(want_e, structure=fp, border_value=0).astype(float))


def test_binary_morph_all_ones_keeps_every_voxel():
    # the reflect / skip boundary does not erode the faces
    v = np.ones((5, 5, 5))
    assert oracle.erode3d(v, "box", 1).sum() == 125


def test_threshold_strict():
    v = np.array([0.5, 0.5000001, 0.4999999, 32768.0, 32769.0]).reshape(1, 1, 5)
    np.testing.assert_array_equal(oracle.threshold(v, 0.5)[0, 0], [0, 1, 0, 1, 1])
    np.testing.assert_array_equal(oracle.threshold(v, 32768.0)[0, 0], [0, 0, 0, 0, 1])


# ----------------------------------------------------------- morph gradients

def _brute_first_arg(v, op, se, r):
    nz, ny, nx = v.shape
    arg = np.zeros(v.shape, dtype=np.int64)
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        best, bi = None, None
        for a in range(-r, r + 1):
            for b in range(-r, r + 1):
                for c in range(-r, r + 1):
                    if se == "ball" and a * a + b * b + c * c > r * r:
                        continue
                    zz, yy, xx = z + a, y + b, x + c
                    if not (0 <= zz < nz and 0 <= yy < ny and 0 <= xx < nx):
                        continue
                    s = v[zz, yy, xx]
                    if best is None or (s > best if op == "dilate" else s < best):
                        best, bi = s, (zz * ny + yy) * nx + xx
        arg[z, y, x] = bi
    return arg


@pytest.mark.parametrize("op", ["erode", "dilate"])
@pytest.mark.parametrize("se,r", [("box", 1), ("ball", 2)])
def test_arg_first_extremum_with_ties(op, se, r):
    v = _rng(15).integers(0, 3, size=(4, 5, 6)).astype(float)  # many ties
    _, arg = oracle.morph3d(v, op, se, r, return_arg=True)
    np.testing.assert_array_equal(arg, _brute_first_arg(v, op, se, r))


@pytest.mark.parametrize("op", ["erode", "dilate"])
def test_morph_backward_matches_finite_difference(op):
    rng = _rng(16)
    v = rng.permutation(6 * 7 * 8).reshape(6, 7, 8).astype(float)  # no ties
    g = rng.standard_normal(v.shape)
    gin = oracle.morph3d_backward(v, g, op, "box", 2)
    h = 1e-3
    for j in rng.choice(v.size, 20, replace=False):
        e = np.zeros(v.size)
        e[j] = h
        e = e.reshape(v.shape)
        fd = (np.sum(g * oracle.morph3d(v + e, op, "box", 2))
              - np.sum(g * oracle.morph3d(v - e, op, "box", 2))) / (2 * h)
        assert gin.reshape(-1)[j] == pytest.approx(fd, rel=1e-9, abs=1e-9)


def test_composite_loss_gradient_matches_central_fd():
    # L = sum c * dilate_box5(G_sigma x), sigma = 1.5, r held at 5.  L is only
    # piecewise smooth (the dilation's argmax switches), so a central
    # difference is valid only if the routing is the same at both ends: start
    # at h = 1e-3 and shrink h until no argmax switches inside [-h, h].
    rng = _rng(17)
    x = rng.standard_normal((10, 11, 12))
    c = rng.standard_normal(x.shape)
    sigma = 1.5
    loss, gx, gs, _ = oracle.gauss_dilate_loss_grad(x, c, sigma, "box", 2)

    def L(xx, ss):
        return oracle.gauss_dilate_loss_grad(xx, c, ss, "box", 2, gauss_radius_fixed=5)[0]

    def args(xx, ss):
        y = oracle.gaussian3d(xx, ss, radius=5, method="separable")
        return oracle.morph3d(y, "dilate", "box", 2, return_arg=True)[1]

    a0 = args(x, sigma)

    def fd(step):
        for h in (1e-3, 3e-4, 1e-4, 3e-5, 1e-5, 3e-6, 1e-6):
            xp, sp = step(+h)
            xm, sm = step(-h)
            if np.array_equal(args(xp, sp), a0) and np.array_equal(args(xm, sm), a0):
                return (L(xp, sp) - L(xm, sm)) / (2 * h)
        pytest.fail("no kink-free step found")

    for k in range(3):
        d = rng.standard_normal(x.shape)
        got = fd(lambda h: (x + h * d, sigma))
        assert float(np.sum(gx * d)) == pytest.approx(got, rel=1e-6, abs=1e-8)
    got_s = fd(lambda h: (x, sigma + h))
    assert gs == pytest.approx(got_s, rel=1e-6, abs=1e-8)


# ------------------------------------------------------------ mean, unsharp

@pytest.mark.parametrize("shape,r", [((9, 11, 13), 1), ((7, 6, 12), (2, 1, 3)), ((3, 4, 5), 3), ((5, 6, 7), (0, 1, 2))])
def test_mean_equals_scipy_uniform(shape, r):
    v = _rng(60).normal(size=shape)
    rz, ry, rx = (r, r, r) if np.ndim(r) == 0 else r
    want = ndi.uniform_filter(v, size=(2 * rz + 1, 2 * ry + 1, 2 * rx + 1), mode="reflect")
    np.testing.assert_allclose(oracle.mean3d(v, r), want, rtol=0, atol=1e-12)


def test_mean_brute_force_tiny():
    # explicit window averages over a symmetric numpy pad (not the oracle's reflect)
    v = _rng(61).normal(size=(4, 5, 3))
    r = (1, 2, 1)
    p = np.pad(v, [(r[0], r[0]), (r[1], r[1]), (r[2], r[2])], mode="symmetric")
    want = np.empty_like(v)
    for z, y, x in itertools.product(*[range(n) for n in v.shape]):
        want[z, y, x] = p[z:z + 2 * r[0] + 1, y:y + 2 * r[1] + 1, x:x + 2 * r[2] + 1].mean()
    np.testing.assert_allclose(oracle.mean3d(v, r), want, rtol=0, atol=1e-13)
    np.testing.assert_allclose(oracle.mean3d(v, r, method="separable"), want, rtol=0, atol=1e-13)


def test_mean_keeps_constant_and_interior_affine():
    np.testing.assert_allclose(oracle.mean3d(np.full((6, 7, 8), 2.5), 2), 2.5, rtol=0, atol=1e-14)
    z, y, x = np.meshgrid(np.arange(12.0), np.arange(13.0), np.arange(14.0), indexing="ij")
    ramp = 0.3 * z - 1.1 * y + 0.7 * x + 2.0
    out = oracle.mean3d(ramp, 2)
    np.testing.assert_allclose(out[2:-2, 2:-2, 2:-2], ramp[2:-2, 2:-2, 2:-2], rtol=0, atol=1e-12)
    assert np.abs(out[0] - ramp[0]).max() > 0.1  # the reflect boundary does bend a ramp


@pytest.mark.parametrize("sigma,amount", [(1.0, 0.5), (1.5, 1.5), ((1.0, 2.0, 0.7), 0.8)])
def test_unsharp_equals_scipy(sigma, amount):
    v = _rng(62).normal(size=(10, 12, 14))
    blur = ndi.gaussian_filter(v, sigma if np.ndim(sigma) else (sigma,) * 3, mode="reflect", truncate=3.0)
    want = v + amount * (v - blur)
    np.testing.assert_allclose(oracle.unsharp3d(v, sigma, amount), want, rtol=0, atol=1e-12)


def test_unsharp_invariants():
    v = _rng(63).normal(size=(8, 9, 10))
    np.testing.assert_allclose(oracle.unsharp3d(v, 1.2, 0.0), v, rtol=0, atol=0)
    np.testing.assert_allclose(oracle.unsharp3d(np.full((6, 6, 6), -1.5), 1.0, 2.0), -1.5, rtol=0, atol=1e-13)
    # a symmetric normalised stencil keeps affine functions away from the faces
    z, y, x = np.meshgrid(np.arange(16.0), np.arange(15.0), np.arange(17.0), indexing="ij")
    ramp = 0.5 * z + 0.25 * y - 0.75 * x
    out = oracle.unsharp3d(ramp, 1.0, 1.3)
    np.testing.assert_allclose(out[3:-3, 3:-3, 3:-3], ramp[3:-3, 3:-3, 3:-3], rtol=0, atol=1e-12)
    # linear in the input
    w = _rng(64).normal(size=v.shape)
    np.testing.assert_allclose(oracle.unsharp3d(2 * v - w, 1.0, 0.7),
                               2 * oracle.unsharp3d(v, 1.0, 0.7) - oracle.unsharp3d(w, 1.0, 0.7), rtol=0, atol=1e-12)


# --------------------------------------------------------- Sobel / Prewitt

@pytest.mark.parametrize("kind", ["sobel", "prewitt"])
@pytest.mark.parametrize("shape", [(7, 9, 11), (3, 1, 5), (1, 1, 4)])
def test_edge_equals_scipy(kind, shape):
    v = _rng(70).normal(size=shape)
    op = ndi.sobel if kind == "sobel" else ndi.prewitt
    for a, got in enumerate(oracle.edge3d_axes(v, kind)):
        np.testing.assert_allclose(got, op(v, axis=a, mode="reflect"), rtol=0, atol=1e-12)
    want = ndi.generic_gradient_magnitude(v, op, mode="reflect")
    np.testing.assert_allclose(oracle.edge3d(v, kind), want, rtol=0, atol=1e-12)


@pytest.mark.parametrize("kind,gain", [("sobel", 32.0), ("prewitt", 18.0)])
def test_edge_constant_and_ramp_closed_form(kind, gain):
    np.testing.assert_allclose(oracle.edge3d(np.full((5, 6, 7), 3.0), kind), 0.0, rtol=0, atol=1e-13)
    # interior of an affine ramp: each axis responds 2 * slope * (sum of the
    # two smoothing kernels' weights: 4 * 4 Sobel, 3 * 3 Prewitt)
    z, y, x = np.meshgrid(np.arange(8.0), np.arange(9.0), np.arange(10.0), indexing="ij")
    a, b, c = 0.5, -1.25, 2.0
    out = oracle.edge3d(a * z + b * y + c * x, kind)
    np.testing.assert_allclose(out[1:-1, 1:-1, 1:-1], gain * math.sqrt(a * a + b * b + c * c), rtol=1e-13)


def test_edge_brute_force_tiny():
    v = _rng(71).normal(size=(3, 4, 5))
    p = np.pad(v, 1, mode="symmetric")
    sm = np.array([1.0, 2.0, 1.0])
    d = np.array([-1.0, 0.0, 1.0])
    want = np.empty_like(v)
    for z, y, x in itertools.product(*[range(n) for n in v.shape]):
        w = p[z:z + 3, y:y + 3, x:x + 3]
        gz = np.einsum("i,j,k,ijk->", d, sm, sm, w)
        gy = np.einsum("i,j,k,ijk->", sm, d, sm, w)
        gx = np.einsum("i,j,k,ijk->", sm, sm, d, w)
        want[z, y, x] = math.sqrt(gz * gz + gy * gy + gx * gx)
    np.testing.assert_allclose(oracle.edge3d(v, "sobel"), want, rtol=0, atol=1e-12)


# ----------------------------------------------------------------- Hessian

@pytest.mark.parametrize("sigma", [1.0, 1.6, (1.0, 2.0, 0.8)])
def test_hessian_equals_scipy(sigma):
    v = _rng(80).normal(size=(11, 12, 13))
    got = oracle.hessian3d(v, sigma)
    for c, (a, b) in enumerate(oracle.HESSIAN_PAIRS):
        order = [0, 0, 0]
        order[a] += 1
        order[b] += 1
        want = ndi.gaussian_filter(v, sigma, order=order, mode="reflect", truncate=3.0)
        np.testing.assert_allclose(got[c], want, rtol=0, atol=1e-12, err_msg=str((a, b)))


def test_hessian_parity_under_flips():
    # even-order components commute with a flip of an axis; components odd
    # in that axis change sign
    v = _rng(81).normal(size=(9, 10, 11))
    h = oracle.hessian3d(v, 1.2)
    for axis in range(3):
        hf = oracle.hessian3d(np.flip(v, axis), 1.2)
        for c, (a, b) in enumerate(oracle.HESSIAN_PAIRS):
            sign = -1.0 if (a == axis) != (b == axis) else 1.0
            np.testing.assert_allclose(hf[c], sign * np.flip(h[c], axis), rtol=0, atol=1e-12)


def test_deriv_taps_moments():
    # sampled derivative taps (M2 = sum k^2 w_k of the normalised taps):
    # order 1 is odd with sum k c_k = M2 / s^2, order 2 is even with
    # sum c_k = (M2 - s^2) / s^4
    for sigma in (1.0, 2.0, 3.5):
        r = oracle.gauss_radius(sigma)
        k = np.arange(-r, r + 1.0)
        w = oracle.gauss_taps(sigma, r)
        m2 = np.sum(k * k * w)
        c1 = oracle.gauss_deriv_taps(sigma, r, 1)
        c2 = oracle.gauss_deriv_taps(sigma, r, 2)
        np.testing.assert_allclose(c1, -c1[::-1], rtol=0, atol=0)
        np.testing.assert_allclose(np.sum(k * c1), m2 / sigma ** 2, rtol=1e-14)
        np.testing.assert_allclose(c2, c2[::-1], rtol=0, atol=0)
        np.testing.assert_allclose(np.sum(c2), (m2 - sigma ** 2) / sigma ** 4, rtol=1e-12, atol=1e-15)
        # truncation at 3 sigma keeps M2 within 1.5 % of s^2, so the
        # derivative of a unit ramp is close to 1
        assert abs(np.sum(k * c1) - 1.0) < 1.5e-2


# -------------------------------------------------------- local thresholds

@pytest.mark.parametrize("method", ["mean", "niblack", "sauvola", "gaussian"])
def test_local_threshold_equals_scipy_statistics(method):
    v = _rng(90).uniform(0, 200, size=(9, 10, 11))
    r, k, R, c = 2, -0.2 if method == "niblack" else 0.3, 100.0, 3.0
    out, t = oracle.local_threshold3d(v, method, radius=r, sigma=1.5, k=k, r_param=R, offset=c, return_t=True)
    m = ndi.uniform_filter(v, size=2 * r + 1, mode="reflect")
    sd = np.sqrt(np.maximum(ndi.uniform_filter(v * v, size=2 * r + 1, mode="reflect") - m * m, 0))
    want = {"mean": m - c, "niblack": m + k * sd, "sauvola": m * (1 + k * (sd / R - 1)),
            "gaussian": ndi.gaussian_filter(v, 1.5, mode="reflect", truncate=3.0) - c}[method]
    np.testing.assert_allclose(t, want, rtol=1e-12, atol=1e-9)
    np.testing.assert_array_equal(out, (v > want).astype(np.uint8))


def test_local_threshold_closed_forms():
    # constant volume: s = 0, so Niblack's T equals v (strict: all 0), the
    # mean threshold with a positive offset keeps everything, Sauvola with
    # 0 < k < 1 keeps a positive constant
    c = np.full((5, 6, 7), 40.0)
    assert oracle.local_threshold3d(c, "niblack", 2, k=-0.2).sum() == 0
    assert oracle.local_threshold3d(c, "mean", 2, offset=1.0).all()
    assert oracle.local_threshold3d(c, "sauvola", 2, k=0.5, r_param=128.0).all()
    # a single bright voxel in a dark box: above the local mean there only
    v = np.zeros((7, 7, 7))
    v[3, 3, 3] = 100.0
    out = oracle.local_threshold3d(v, "mean", 1)
    assert out.sum() == 1 and out[3, 3, 3] == 1
    # box standard deviation of a two-valued window, by hand
    w = np.zeros((3, 3, 3))
    w[0] = 27.0  # one face of 9 voxels at 27, the rest 0: m = 9, s = sqrt(243 - 81)
    _, t = oracle.local_threshold3d(w, "niblack", 1, k=1.0, return_t=True)
    assert abs(t[1, 1, 1] - (9.0 + math.sqrt(162.0))) < 1e-12


# -------------------------------------------------------------------- Otsu

def test_otsu_minimises_within_class_variance_brute_force():
    # Otsu's split maximises the between-class variance, which is the same as
    # minimising the within-class variance computed from the values directly
    rng = _rng(100)
    v = np.concatenate([rng.normal(60, 8, 3000), rng.normal(170, 15, 2000)]).clip(0, 255).astype(np.int64)
    k = oracle.otsu_threshold(v, 256)
    best_k, best = None, None
    for t in range(255):
        a, b = v[v <= t], v[v > t]
        if len(a) == 0 or len(b) == 0:
            continue
        w = len(a) * a.var() + len(b) * b.var()
        if best is None or w < best - 1e-9 * abs(best):
            best, best_k = w, t
    # ties in the within-class form may pick a neighbouring empty bin: the
    # two splits must put every voxel in the same class
    assert np.array_equal(v > k, v > best_k)


def test_otsu_hand_worked():
    # two values: every split between them is optimal; the first one wins
    v = np.array([3, 3, 3, 10, 10])
    assert oracle.otsu_threshold(v, 16) == 3
    np.testing.assert_array_equal(oracle.otsu3d(v, 16), [0, 0, 0, 1, 1])
    assert oracle.otsu_threshold(np.full(7, 5), 16) == -1
    # three equal clusters at 0, 10, 20: the variance of a split {0} | {10, 20}
    # (1 * 2 * (0 - 15)^2 = 450 per triple) equals {0, 10} | {20}: first wins
    assert oracle.otsu_threshold(np.repeat([0, 10, 20], 4), 32) == 0
