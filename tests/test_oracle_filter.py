"""Pins for the oracle's regional reconstruction filter, its adjoint and the loss seed (no GPU).

The filter's functional form is a reading of the paper (Gaussian h_j truncated to the
window, width from the region of the output pixel, border clipped and renormalised); these
tests pin the oracle's arithmetic to that reading by brute force, invariants, closed forms
and finite differences.
"""

import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle.regional_filter import filter_backward, filter_forward, mse_loss_seed, region_index


# ----------------------------------------------------------------------------- region map
@pytest.mark.parametrize("n_regions", [1, 2, 3, 5, 7, 20, 25])
def test_region_map_matches_pixel_centre_cells(n_regions):
    # A pixel belongs to grid cell floor(N * c) of its raster-space centre c = (x + 1/2) / W.
    for W in list(range(1, 41)) + [96, 1920]:
        H = max(1, (W * 3) // 5)
        k = region_index(W, H, n_regions)
        for x in range(W):
            cx = Fraction(2 * x + 1, 2 * W)
            assert k[0, x] % n_regions == math.floor(n_regions * cx)
        for y in range(H):
            cy = Fraction(2 * y + 1, 2 * H)
            assert k[y, 0] // n_regions == math.floor(n_regions * cy)
    assert region_index(1920, 1080, 20).max() == 399


def test_single_region_grid_maps_everything_to_zero():
    assert np.all(region_index(37, 23, 1) == 0)


# ----------------------------------------------------------------------------- forward
def _brute_forward(mean, lam, n_regions, r, lam_min):
    """Literal loops over output pixels and their windows."""
    C, H, W = mean.shape
    out = np.zeros((C, H, W))
    for y in range(H):
        for x in range(W):
            kx = (2 * x + 1) * n_regions // (2 * W)
            ky = (2 * y + 1) * n_regions // (2 * H)
            s2 = math.exp(max(float(lam[ky * n_regions + kx]), lam_min))
            num = [0.0] * C
            den = 0.0
            for py in range(y - r, y + r + 1):
                for px in range(x - r, x + r + 1):
                    if 0 <= px < W and 0 <= py < H:
                        h = math.exp(-((px - x) ** 2 + (py - y) ** 2) / (2 * s2))
                        den += h
                        for c in range(C):
                            num[c] += h * mean[c, py, px]
            for c in range(C):
                out[c, y, x] = num[c] / den
    return out


def _scatter_forward(mean, lam, n_regions, r, lam_min):
    """Splat form: every source pixel p adds its weighted value into each output j whose
    window contains it."""
    C, H, W = mean.shape
    k = region_index(W, H, n_regions)
    s2 = np.exp(np.maximum(lam.astype(np.float64), lam_min))[k]
    num = np.zeros((C, H, W))
    den = np.zeros((H, W))
    for py in range(H):
        for px in range(W):
            for y in range(max(0, py - r), min(H, py + r + 1)):
                for x in range(max(0, px - r), min(W, px + r + 1)):
                    h = math.exp(-((px - x) ** 2 + (py - y) ** 2) / (2 * s2[y, x]))
                    den[y, x] += h
                    num[:, y, x] += h * mean[:, py, px]
    return num / den


@pytest.mark.parametrize("W,H,N,r", [(9, 7, 3, 2), (6, 11, 4, 3), (5, 4, 2, 6), (1, 1, 1, 2), (13, 3, 5, 1)])
def test_forward_brute_force_and_scatter(W, H, N, r):
    rng = np.random.default_rng(W * 100 + H)
    mean = rng.random((3, H, W)) * 2 - 0.3
    lam = rng.uniform(-2.0, 2.5, N * N)
    lam[0] = -40.0  # below the clamp
    out, _ = filter_forward(mean, lam, N, r, -30.0)
    ref = _brute_forward(mean, lam, N, r, -30.0)
    np.testing.assert_allclose(out, ref, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(_scatter_forward(mean, lam, N, r, -30.0), ref, rtol=1e-13, atol=1e-14)


def test_constant_image_unchanged_and_weights_normalised():
    rng = np.random.default_rng(1)
    lam = rng.uniform(-1, 3, 16)
    mean = np.full((3, 10, 12), 0.7)
    out, den = filter_forward(mean, lam, 4, 5)
    np.testing.assert_allclose(out, 0.7, rtol=1e-14)
    ones, _ = filter_forward(np.ones((1, 10, 12)), lam, 4, 5)
    np.testing.assert_allclose(ones, 1.0, rtol=1e-14)
    assert np.all(den >= 1.0)  # the centre tap has weight exactly 1


def test_lambda_min_is_identity():
    rng = np.random.default_rng(2)
    mean = rng.random((3, 8, 9))
    out, den = filter_forward(mean, np.full(9, -30.0), 3, 4, -30.0)
    assert np.array_equal(out, mean)
    assert np.all(den == 1.0)
    out2, _ = filter_forward(mean, np.full(9, -55.0), 3, 4, -30.0)
    assert np.array_equal(out2, mean)


def test_affine_image_reproduced_in_interior():
    H, W, r = 20, 24, 3
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    mean = np.stack([0.3 + 0.02 * x - 0.01 * y, 1.0 - 0.03 * y, 0.5 * np.ones_like(x)])
    lam = np.linspace(-1.0, 2.0, 16)
    out, _ = filter_forward(mean, lam, 4, r)
    np.testing.assert_allclose(out[:, r:H - r, r:W - r], mean[:, r:H - r, r:W - r], rtol=1e-13)


def test_quadratic_image_gains_kernel_second_moment():
    # mean = x^2: interior output = x^2 + sum_dx w(dx) dx^2 / sum_dx w(dx) with the 1-D
    # weights w(d) = exp(-d^2 / (2 sigma_j^2)) of the OUTPUT pixel's region.
    H, W, r, N = 18, 30, 4, 3
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    mean = (x * x)[None]
    lam = np.array([-1.0, 0.0, 0.5, 1.0, 1.5, 2.0, 2.5, 3.0, -0.5])
    out, _ = filter_forward(mean, lam, N, r)
    for yy in range(r, H - r):
        for xx in range(r, W - r):
            k = ((2 * yy + 1) * N // (2 * H)) * N + (2 * xx + 1) * N // (2 * W)
            s2 = math.exp(lam[k])
            w = [math.exp(-d * d / (2 * s2)) for d in range(-r, r + 1)]
            m2 = sum(wi * d * d for wi, d in zip(w, range(-r, r + 1))) / sum(w)
            assert out[0, yy, xx] == pytest.approx(xx * xx + m2, rel=1e-13)


def test_separable_equals_two_dimensional_window():
    # With one region the clipped Gaussian window factorises: rows, then columns.
    rng = np.random.default_rng(4)
    H, W, r = 11, 14, 3
    mean = rng.random((2, H, W))
    lam = np.array([0.7])
    out, _ = filter_forward(mean, lam, 1, r)
    s2 = math.exp(0.7)
    w = np.array([math.exp(-d * d / (2 * s2)) for d in range(-r, r + 1)])

    def conv1d(a, axis):
        n = a.shape[axis]
        num = np.zeros_like(a)
        den = np.zeros(n)
        for i in range(n):
            for t, d in enumerate(range(-r, r + 1)):
                j = i + d
                if 0 <= j < n:
                    den[i] += w[t]
                    src = np.take(a, j, axis=axis)
                    idx = [slice(None)] * a.ndim
                    idx[axis] = i
                    num[tuple(idx)] += w[t] * src
        shape = [1] * a.ndim
        shape[axis] = n
        return num / den.reshape(shape)

    sep = conv1d(conv1d(mean, 2), 1)
    np.testing.assert_allclose(out, sep, rtol=1e-13)


# ----------------------------------------------------------------------------- loss seed
def test_loss_seed_closed_form_and_gradient():
    rng = np.random.default_rng(5)
    out = rng.random((3, 4, 5))
    ref = rng.random((3, 4, 5))
    L, U = mse_loss_seed(out, ref)
    assert L == pytest.approx(((out - ref) ** 2).sum() / 60.0, rel=1e-15)
    eps = 1e-6
    for idx in [(0, 0, 0), (2, 3, 4), (1, 2, 1)]:
        o1 = out.copy()
        o1[idx] += eps
        o2 = out.copy()
        o2[idx] -= eps
        fd = (mse_loss_seed(o1, ref)[0] - mse_loss_seed(o2, ref)[0]) / (2 * eps)
        assert U[idx] == pytest.approx(fd, rel=1e-7)


# ----------------------------------------------------------------------------- backward
def _brute_backward(U, mean, lam, n_regions, r, lam_min, S):
    C, H, W = mean.shape
    G = np.zeros((C, H, W))
    gl = np.zeros(n_regions * n_regions)
    out = _brute_forward(mean, lam, n_regions, r, lam_min)
    for y in range(H):
        for x in range(W):
            k = ((2 * y + 1) * n_regions // (2 * H)) * n_regions + (2 * x + 1) * n_regions // (2 * W)
            s2 = math.exp(max(float(lam[k]), lam_min))
            live = float(lam[k]) >= lam_min
            taps = []
            for py in range(y - r, y + r + 1):
                for px in range(x - r, x + r + 1):
                    if 0 <= px < W and 0 <= py < H:
                        d2 = (px - x) ** 2 + (py - y) ** 2
                        taps.append((py, px, d2, math.exp(-d2 / (2 * s2))))
            D = sum(t[3] for t in taps)
            for py, px, d2, h in taps:
                for c in range(C):
                    G[c, py, px] += U[c, y, x] * h / D / S
                    if live:
                        gl[k] += U[c, y, x] * h * d2 / (2 * s2) * (mean[c, py, px] - out[c, y, x]) / D
    return G, gl, out


@pytest.mark.parametrize("W,H,N,r,S", [(9, 7, 3, 2, 4), (7, 10, 2, 3, 1), (4, 3, 2, 5, 3)])
def test_backward_brute_force(W, H, N, r, S):
    rng = np.random.default_rng(W + 7 * H)
    mean = rng.random((3, H, W))
    U = rng.standard_normal((3, H, W))
    lam = rng.uniform(-1.5, 2.0, N * N)
    lam[-1] = -31.0  # clamped region: no lambda gradient
    out, _ = filter_forward(mean, lam, N, r)
    G, gl = filter_backward(U, mean, out, lam, N, r, -30.0, S)
    Gb, glb, outb = _brute_backward(U, mean, lam, N, r, -30.0, S)
    np.testing.assert_allclose(out, outb, rtol=1e-13)
    np.testing.assert_allclose(G, Gb, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(gl, glb, rtol=1e-11, atol=1e-15)
    assert gl[-1] == 0.0


def _loss_of(radiance, lam, ref, N, r, lam_min=-30.0):
    st = oracle.stats_accumulate(radiance, None, 0)
    out, _ = filter_forward(st["mean"], lam, N, r, lam_min)
    return mse_loss_seed(out, ref)[0]


def test_backward_matches_central_differences():
    # Tiny frame: 9 x 7, S = 4, r = 2, N = 3; FP64 central differences, step 1e-6.
    rng = np.random.default_rng(9)
    W, H, S, N, r = 9, 7, 4, 3, 2
    rad = rng.random((3, S, H, W))
    ref = rng.random((3, H, W))
    lam = rng.uniform(-1.0, 1.5, N * N)
    st = oracle.stats_accumulate(rad, None, 0)
    out, _ = filter_forward(st["mean"], lam, N, r)
    _, U = mse_loss_seed(out, ref)
    G, gl = filter_backward(U, st["mean"], out, lam, N, r, -30.0, S)
    eps = 1e-6
    for k in range(N * N):
        lp = lam.copy()
        lp[k] += eps
        lm = lam.copy()
        lm[k] -= eps
        fd = (_loss_of(rad, lp, ref, N, r) - _loss_of(rad, lm, ref, N, r)) / (2 * eps)
        assert gl[k] == pytest.approx(fd, rel=1e-6, abs=1e-10)
    for (c, s, y, x) in [(0, 0, 0, 0), (1, 3, 6, 8), (2, 1, 3, 4), (0, 2, 5, 1)]:
        rp = rad.copy()
        rp[c, s, y, x] += eps
        rm = rad.copy()
        rm[c, s, y, x] -= eps
        fd = (_loss_of(rp, lam, ref, N, r) - _loss_of(rm, lam, ref, N, r)) / (2 * eps)
        assert G[c, y, x] == pytest.approx(fd, rel=1e-6, abs=1e-11)


def test_backward_is_the_adjoint_of_forward():
    # <U, F v> = <F^T U, v> for the linear map v -> filter_forward(v) at fixed lambda;
    # F^T U is S * G with S = 1.
    rng = np.random.default_rng(12)
    H, W, N, r = 12, 15, 4, 3
    lam = rng.uniform(-1, 2, N * N)
    v = rng.standard_normal((3, H, W))
    U = rng.standard_normal((3, H, W))
    Fv, _ = filter_forward(v, lam, N, r)
    G, _ = filter_backward(U, v, Fv, lam, N, r, -30.0, 1)
    assert (U * Fv).sum() == pytest.approx((G * v).sum(), rel=1e-12)


def test_backward_mass_and_special_cases():
    rng = np.random.default_rng(13)
    H, W, N, r, S = 10, 11, 3, 4, 5
    lam = rng.uniform(-1, 2, N * N)
    U = rng.standard_normal((3, H, W))
    mean = rng.random((3, H, W))
    out, _ = filter_forward(mean, lam, N, r)
    G, _ = filter_backward(U, mean, out, lam, N, r, -30.0, S)
    # sum over pixels and samples of dL/dg equals sum_j U_j (weights sum to one)
    np.testing.assert_allclose((G * S).sum(axis=(1, 2)), U.sum(axis=(1, 2)), rtol=1e-12)
    # constant image: the output cannot depend on lambda
    const = np.full((3, H, W), 0.4)
    out_c, _ = filter_forward(const, lam, N, r)
    _, gl_c = filter_backward(U, const, out_c, lam, N, r, -30.0, S)
    np.testing.assert_allclose(gl_c, 0.0, atol=1e-14)
    # lambda at its minimum: identity filter, G = U / S, no lambda gradient below it
    lam_min = np.full(N * N, -30.0)
    out_m, _ = filter_forward(mean, lam_min, N, r)
    G_m, gl_m = filter_backward(U, mean, out_m, lam_min, N, r, -30.0, S)
    np.testing.assert_allclose(G_m, U / S, rtol=1e-15)
    assert np.all(gl_m == 0.0)


def test_crops_reproduce_the_full_image():
    # a crop keeps the full image's regions and border: results agree where every pixel
    # they read lies in the crop (r from non-image crop edges for out, 2r for G)
    rng = np.random.default_rng(21)
    H, W, N, r, S = 40, 52, 5, 3, 4
    lam = rng.uniform(-1, 2, N * N)
    mean = rng.random((3, H, W))
    ref = rng.random((3, H, W))
    out, D = filter_forward(mean, lam, N, r)
    L, U = mse_loss_seed(out, ref)
    G, gl = filter_backward(U, mean, out, lam, N, r, -30.0, S)
    regions_checked = 0
    for x0, y0, w, h in [(0, 0, 30, 25), (9, 7, 30, 26), (20, 14, 32, 26), (0, 20, 52, 20)]:
        crop = dict(origin=(x0, y0), image_size=(W, H))
        sl = (slice(None), slice(y0, y0 + h), slice(x0, x0 + w))
        out_c, D_c = filter_forward(mean[sl], lam, N, r, **crop)

        def interior(m):  # rows/columns at least m from crop edges that are not image edges
            ys = slice(0 if y0 == 0 else m, h if y0 + h == H else h - m)
            xs = slice(0 if x0 == 0 else m, w if x0 + w == W else w - m)
            return ys, xs

        ys, xs = interior(r)
        np.testing.assert_allclose(out_c[:, ys, xs], out[sl][:, ys, xs], rtol=1e-14, atol=0)
        np.testing.assert_allclose(D_c[ys, xs], D[sl[1:]][ys, xs], rtol=1e-14)
        L_c, U_c = mse_loss_seed(out[sl], ref[sl], count=out.size)
        np.testing.assert_array_equal(U_c, U[sl])
        G_c, gl_c = filter_backward(U[sl], mean[sl], out[sl], lam, N, r, -30.0, S, **crop)
        ys, xs = interior(2 * r)
        np.testing.assert_allclose(G_c[:, ys, xs], G[sl][:, ys, xs], rtol=1e-12, atol=1e-15)
        # regions lying r inside the non-image crop edges
        k = region_index(W, H, N)
        ys, xs = interior(r)
        inner = np.zeros((H, W), bool)
        inner[y0:y0 + h, x0:x0 + w][ys, xs] = True
        full_regions = [kk for kk in range(N * N) if inner[k == kk].all()]
        if x0 == 0 and y0 == 0 and w == W and h == H:
            assert len(full_regions) == N * N
        for kk in full_regions:
            assert gl_c[kk] == pytest.approx(gl[kk], rel=1e-12, abs=1e-15)
        regions_checked += len(full_regions)
    assert regions_checked >= 4
    # the pixel-count override: the crop's share of the loss
    assert mse_loss_seed(out[:, :10], ref[:, :10], count=out.size)[0] < L
    with pytest.raises(ValueError):
        filter_forward(mean, lam, N, r, origin=(1, 0), image_size=(W, H))
