"""NumPy implementation of the synthetic render-buffer recipe (small frames, CPU).

Layout of the returned planes: ``radiance[c][s][y][x]`` (c < 3) and
``features[c][s][y][x]`` (c < 7: albedo rgb, normal xyz, depth), x contiguous.
"""

import numpy as np

from .recipe import (
    SAMPLE_PIXEL,
    MAX_SPP,
    box_muller,
    draw,
    frame_key,
    sample_key,
    scene,
    uniform_pair,
)

NOISE_CONST = 0
NOISE_UNIFORM = 1


def _pixel_grid(W, H, rows=None):
    """x, y and pixel index of rows [y0, y1) of a W x H frame (all rows by default)."""
    y0, y1 = (0, H) if rows is None else rows
    y, x = np.meshgrid(np.arange(y0, y1, dtype=np.uint64), np.arange(W, dtype=np.uint64), indexing="ij")
    return x, y, y * np.uint64(W) + x


def _rows(H, rows):
    y0, y1 = (0, H) if rows is None else (int(rows[0]), int(rows[1]))
    if not 0 <= y0 < y1 <= H:
        raise ValueError("rows outside the frame")
    return y0, y1


def pixel_sigma(W, H, seed, frame=0, noise=NOISE_UNIFORM, sigma=0.1, rows=None):
    """Per-pixel noise scale sigma_p [H, W] (float64); [y1 - y0, W] for rows = (y0, y1)."""
    y0, y1 = _rows(H, rows)
    if noise == NOISE_CONST:
        return np.full((y1 - y0, W), float(sigma))
    _, _, pix = _pixel_grid(W, H, (y0, y1))
    fk = frame_key(seed, frame)
    ua, _ = uniform_pair(draw(sample_key(fk, pix, SAMPLE_PIXEL), 0))
    return 0.02 + 0.48 * ua


def _sample_values(W, H, s, fk, sig, firefly_p, rows=None):
    """Radiance (3,H,W) and features (7,H,W), float64, for sample index s (rows [y0, y1)
    only when given)."""
    x, y, pix = _pixel_grid(W, H, rows)
    sk = sample_key(fk, pix, np.uint64(s))
    xi_x, xi_y = uniform_pair(draw(sk, 0))
    u1, u2 = uniform_pair(draw(sk, 1))
    u3, u4 = uniform_pair(draw(sk, 2))
    uf, _ = uniform_pair(draw(sk, 3))
    u = (x.astype(np.float64) + xi_x) / float(W)
    v = (y.astype(np.float64) + xi_y) / float(H)
    L, alb, nrm, depth = scene(u, v)
    z0, z1 = box_muller(u1, u2)
    z2, z3 = box_muller(u3, u4)
    g = np.stack([L[0] + sig * z0, L[1] + sig * z1, L[2] + sig * z2])
    fire = uf < firefly_p
    if np.any(fire):
        y_ff = np.exp(3.0 + z3)
        g = g + np.where(fire, y_ff, 0.0)[None]
    feats = np.concatenate([alb, nrm, depth[None]], axis=0)
    return g, feats


def make_frame(W, H, S, seed, frame=0, noise=NOISE_UNIFORM, sigma=0.1, firefly_p=1e-3,
               feature_dtype=np.float32, with_features=True, rows=None):
    """Sample planes of one frame.

    Returns ``(radiance float32 [3,S,H,W], features [7,S,H,W] or None)``; with
    ``rows = (y0, y1)`` only those rows of the frame ([.., y1 - y0, W], the same values).
    """
    if not (1 <= S <= MAX_SPP):
        raise ValueError("S out of range")
    y0, y1 = _rows(H, rows)
    fk = frame_key(seed, frame)
    sig = pixel_sigma(W, H, seed, frame, noise, sigma, (y0, y1))
    rad = np.empty((3, S, y1 - y0, W), dtype=np.float32)
    feat = np.empty((7, S, y1 - y0, W), dtype=feature_dtype) if with_features else None
    for s in range(S):
        g, f = _sample_values(W, H, s, fk, sig, firefly_p, (y0, y1))
        rad[:, s] = g.astype(np.float32)
        if with_features:
            # fp16 storage rounds through fp32 (the GPU generator does the same)
            feat[:, s] = f.astype(np.float32).astype(feature_dtype)
    return rad, feat


def make_reference(W, H, seed, frame=0, spp=4096, noise=NOISE_UNIFORM, sigma=0.1, firefly_p=1e-3, rows=None):
    """High-spp reference image [3,H,W] float32: the float64 mean of ``spp`` float32-rounded
    radiance samples drawn from the independent stream ``seed`` (rows [y0, y1) only when
    given)."""
    y0, y1 = _rows(H, rows)
    fk = frame_key(seed, frame)
    sig = pixel_sigma(W, H, seed, frame, noise, sigma, (y0, y1))
    acc = np.zeros((3, y1 - y0, W), dtype=np.float64)
    for s in range(spp):
        g, _ = _sample_values(W, H, s, fk, sig, firefly_p, (y0, y1))
        acc += g.astype(np.float32).astype(np.float64)
    return (acc / float(spp)).astype(np.float32)


def make_lambda(n_regions, seed=99, frame=0, centre=1.0, spread=0.5):
    """Per-region log-variance table lam[n_regions**2] (float32), row-major (ky, kx):
    ``centre + (2u - 1) * spread``."""
    fk = frame_key(seed, frame)
    k = np.arange(n_regions * n_regions, dtype=np.uint64)
    ua, _ = uniform_pair(draw(sample_key(fk, k, 0), 0))
    return (centre + (2.0 * ua - 1.0) * spread).astype(np.float32)


def ar1_samples(C, S, H, W, rho, seed=7):
    """Stationary AR(1) sample sequences a_s = rho a_{s-1} + sqrt(1-rho^2) Z_s, float32
    [C,S,H,W], for tests of the lag statistics (standard normal marginals)."""
    rng = np.random.default_rng(seed)
    out = np.empty((C, S, H, W), dtype=np.float64)
    a = rng.standard_normal((C, H, W))
    c = np.sqrt(1.0 - rho * rho)
    for s in range(S):
        if s > 0:
            a = rho * a + c * rng.standard_normal((C, H, W))
        out[:, s] = a
    return out.astype(np.float32)
