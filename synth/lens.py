"""Seeded inputs for the lens-perturbation chains (no scene or renderer is available):

* make_luminance(W, H, seed): float32 [H, W], the Rec. 709 luminance of the synthetic scene
  (synth.recipe.scene) at the pixel centres, modulated by stripes whose period grows from
  4 px at the top to 64 px at the bottom (local contrast differs from region to region, so
  the adapted scales must too), with a black rectangle (zero density, never entered) and
  0.1 % of pixels 20 times brighter;
* make_lens_chains(n, W, H, tan_half_fov_x, seed): float32 [n, 3] unit primary directions
  through uniform points of the central 96 % of the frame, 0.1 % of them invalid (behind the
  camera or NaN);
* make_lens_noise(n, seed, batch): float32 [n, 3] uniforms (u, v, acceptance), 24 bits each,
  from the counter-based generator of synth.recipe (key: seed, batch, chain).

None of the method's arithmetic is here.
"""

import numpy as np

from .recipe import draw, frame_key, mix64, scene, uniform_pair

GAMMA64 = np.uint64(0x9E3779B97F4A7C15)


def make_luminance(W, H, seed):
    u = (np.arange(W) + 0.5) / W
    v = (np.arange(H) + 0.5) / H
    uu, vv = np.meshgrid(u, v)
    L = scene(uu, vv)[0]
    lum = 0.2126 * L[0] + 0.7152 * L[1] + 0.0722 * L[2]
    x = np.arange(W)[None, :] + 0.5
    period = 4.0 * 2.0 ** (4.0 * vv)
    lum = lum * (1.0 + 0.8 * np.sin(2.0 * np.pi * x / period))
    lum[int(0.8 * H):int(0.9 * H), int(0.05 * W):int(0.15 * W)] = 0.0
    rng = np.random.default_rng([seed, W, H])
    lum = np.where(rng.random((H, W)) < 1e-3, 20.0 * lum, lum)
    return lum.astype(np.float32)


def make_lens_chains(n, W, H, tan_half_fov_x, seed):
    rng = np.random.default_rng([seed, n, 7])
    tx = float(np.float32(tan_half_fov_x))
    ty = tx * H / W
    sx = rng.uniform(0.02, 0.98, n)
    sy = rng.uniform(0.02, 0.98, n)
    d = np.stack([(2.0 * sx - 1.0) * tx, (2.0 * sy - 1.0) * ty, np.ones(n)], axis=1)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    bad = rng.random(n) < 1e-3
    half = rng.random(n) < 0.5
    d[bad & half] = [0.0, 0.0, -1.0]
    d[bad & ~half, 0] = np.nan
    return d.astype(np.float32)


def make_lens_noise(n, seed, batch=0, chunk=1 << 22):
    out = np.empty((n, 3), dtype=np.float32)
    fk = frame_key(seed, batch)
    for s0 in range(0, n, chunk):
        i = np.arange(s0, min(n, s0 + chunk), dtype=np.uint64)
        with np.errstate(over="ignore"):
            key = mix64(np.uint64(fk) + (i + np.uint64(1)) * GAMMA64)
        u1, u2 = uniform_pair(draw(key, 0))
        u3, _ = uniform_pair(draw(key, 1))
        sl = slice(s0, s0 + len(i))
        out[sl, 0] = u1
        out[sl, 1] = u2
        out[sl, 2] = u3
    return out
