"""One Metropolis step of screen-space chains under the regional adaptive lens perturbation
(Sec. 3.3 "Lens Perturbation" and "Perturbing Ray Directions"; Sec. 6.1 "2d Partition for
the Lens Perturbation"; Alg. 1 lines 8-13), with the image's luminance standing in for the
path contribution. NumPy.

TEST INFRASTRUCTURE (see the package docstring): only tests/, smoke() and bench.py's
cpu_baseline leg may use it.

Reading (no renderer here): the state of a chain is its primary ray direction omega of a
pinhole camera looking along +z. Its raster position in canonical screen space [0, 1)^2 is

    sx = 1/2 + (1/2) (omega_x / omega_z) / tx,   sy = 1/2 + (1/2) (omega_y / omega_z) / ty,

tx = tan of half the horizontal field of view, ty = tx H / W (rounded once from fp64); the
state is in the frame iff omega_z > 0 and both lie in [0, 1); its pixel is
(min(floor(sx W), W - 1), min(floor(sy H), H - 1)) and its region the screen-grid cell of that
pixel (the filter's map, Sec. 6.1). The target density over directions is the luminance of
the pixel, pi(omega) = L[pixel], zero outside the frame. The proposal perturbs omega with
sigma_k of the current region (oracle.direction_sampler; its density depends only on the
angle between omega and omega', so it is symmetric), and the acceptance probability is
alpha = min(1, pi(omega') / pi(omega)); the chain moves iff its uniform is below alpha.
A proposal outside the frame has alpha = 0 (rejected at once, as a lens perturbation that
hits an invalid vertex is). A chain whose state is outside the frame (or NaN) has no region
(-1) and alpha NaN, and does not move.

Precision: the raster map and every decision (pixel, region, alpha, accept) are taken in
float32, one IEEE operation at a time in the order written above, as the kernel takes them;
omega' is the direction sampler's fp64 proposal rounded to float32.
"""

import numpy as np

from . import direction_sampler as ds
from .regional_filter import region_index

F32 = np.float32


def tan_half_y(tan_half_x, W, H):
    """ty = tx H / W, from fp64 rounded to float32."""
    return F32(float(F32(tan_half_x)) * H / W)


def raster(omega, W, H, tan_half_x):
    """(inside [n] bool, ix [n], iy [n]) of float32 directions [n, 3]."""
    w = np.asarray(omega, dtype=F32)
    tx = F32(tan_half_x)
    ty = tan_half_y(tan_half_x, W, H)
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        qx = w[:, 0] / w[:, 2]
        qy = w[:, 1] / w[:, 2]
        sx = F32(0.5) + F32(0.5) * (qx / tx)
        sy = F32(0.5) + F32(0.5) * (qy / ty)
        inside = (w[:, 2] > 0) & (sx >= 0) & (sx < 1) & (sy >= 0) & (sy < 1)
        px = np.where(inside, sx * F32(W), F32(0))
        py = np.where(inside, sy * F32(H), F32(0))
    ix = np.minimum(px.astype(np.int64), W - 1)
    iy = np.minimum(py.astype(np.int64), H - 1)
    return inside, ix, iy


def sort_tile_side(W, H, max_tiles=63):
    """Side T of the screen tiles of the chain reorder: the smallest power of two >= 16 with
    ceil(W / T) * ceil(H / T) <= max_tiles."""
    T = 16
    while -(-W // T) * -(-H // T) > max_tiles:
        T *= 2
    return T


def tile_order(omega, W, H, tan_half_x):
    """The chain reorder (not an operation of the paper: the chains are independent, so their
    order in memory is free). Key of chain i: the T x T tile of its pixel under the raster map
    above, row-major, or the tile count for a chain outside the frame; the chains sorted by key,
    stably. Returns (keys int64 [n], perm int64 [n]) with perm the old index of each chain in
    the new order."""
    inside, ix, iy = raster(omega, W, H, tan_half_x)
    T = sort_tile_side(W, H)
    ntx, nty = -(-W // T), -(-H // T)
    keys = np.where(inside, (iy // T) * ntx + ix // T, ntx * nty)
    return keys, np.argsort(keys, kind="stable")


def step(luminance, tan_half_x, lam, n_regions, omega, noise):
    """One step of every chain. luminance [H, W] float32; lam [n_regions^2] (float64);
    omega [n, 3] float32 states; noise [n, 3] = (u, v, u_accept). Returns
    (omega_next float32 [n, 3], region int64 [n], alpha float32 [n], omega_prop float32 [n, 3])."""
    L = np.asarray(luminance, dtype=F32)
    H, W = L.shape
    omega = np.asarray(omega, dtype=F32)
    noise = np.asarray(noise, dtype=F32)
    n = omega.shape[0]
    inside, ix, iy = raster(omega, W, H, tan_half_x)
    kmap = region_index(W, H, n_regions)
    region = np.where(inside, kmap[iy, ix], -1)
    prop64, _ = ds.perturb_directions(lam, region, omega.astype(np.float64), noise[:, :2].astype(np.float64))
    prop = prop64.astype(F32)
    alpha = acceptance(L, tan_half_x, omega, prop)
    accept = noise[:, 2] < alpha
    nxt = np.where(accept[:, None], prop, omega)
    prop = np.where(inside[:, None], prop, F32(np.nan))
    assert nxt.shape == (n, 3)
    return nxt, region, alpha, prop


def ratio(new, cur):
    """alpha = min(1, new / cur) of luminances (float32): 1 if new >= cur, else the quotient."""
    new = np.asarray(new, dtype=F32)
    cur = np.asarray(cur, dtype=F32)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(new >= cur, F32(1), new / cur).astype(F32)


def acceptance(luminance, tan_half_x, omega, prop):
    """alpha of moving from each state omega [n, 3] to its proposal prop [n, 3] (float32):
    NaN for a state outside the frame, 0 for a proposal outside it, else
    min(1, pi(prop) / pi(omega)) with pi the luminance of the pixel."""
    L = np.asarray(luminance, dtype=F32)
    H, W = L.shape
    omega = np.asarray(omega, dtype=F32)
    prop = np.asarray(prop, dtype=F32)
    inside, ix, iy = raster(omega, W, H, tan_half_x)
    inside2, ix2, iy2 = raster(np.where(inside[:, None], prop, F32(0)), W, H, tan_half_x)
    inside2 &= inside
    cur = L[iy, ix]
    new = np.where(inside2, L[iy2, ix2], F32(0))
    alpha = np.where(inside2, ratio(new, cur), F32(0)).astype(F32)
    return np.where(inside, alpha, F32(np.nan)).astype(F32)


def pixel_solid_angles(W, H, tan_half_x):
    """Solid angle of every pixel [H, W] seen from the pinhole (image plane at z = 1): for a
    rectangle [x0, x1] x [y0, y1], F(x1, y1) - F(x0, y1) - F(x1, y0) + F(x0, y0) with
    F(x, y) = atan(x y / sqrt(1 + x^2 + y^2))."""
    tx = float(F32(tan_half_x))
    ty = float(tan_half_y(tan_half_x, W, H))
    xe = (2.0 * np.arange(W + 1) / W - 1.0) * tx
    ye = (2.0 * np.arange(H + 1) / H - 1.0) * ty
    X, Y = np.meshgrid(xe, ye)
    F = np.arctan2(X * Y, np.sqrt(1.0 + X * X + Y * Y))
    return F[1:, 1:] - F[1:, :-1] - F[:-1, 1:] + F[:-1, :-1]


def pixel_centre_directions(W, H, tan_half_x):
    """Unit directions through the pixel centres, float32 [H * W, 3] in row-major order."""
    tx = float(F32(tan_half_x))
    ty = float(tan_half_y(tan_half_x, W, H))
    xs = (2.0 * (np.arange(W) + 0.5) / W - 1.0) * tx
    ys = (2.0 * (np.arange(H) + 0.5) / H - 1.0) * ty
    X, Y = np.meshgrid(xs, ys)
    d = np.stack([X.ravel(), Y.ravel(), np.ones(W * H)], axis=1)
    return (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(F32)
