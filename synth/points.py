"""Seeded stand-in for the chain states an MLT renderer looks up in a quadtree partition
(the paper's renderer and scenes are not available).

Point i of batch b is (root, x, y): the tree it belongs to and its coordinates in that
tree's unit square. For the 2-D partition (one tree) x, y is the raster position of the
state's primary vertex; for the 4-D partition the root is the screen grid cell and x, y are
the two coordinates of the outgoing direction.

* with probability 1/2 the point lies in a bright spot: a normal blob of standard deviation
  0.03 around (0.3, 0.7) or (0.8, 0.2) (one of the two with equal chance), clamped to the
  unit square; otherwise x = u^3, y = u' (density falling off to the right), so the
  partition has to refine strongly in some places and hardly in others;
* root = floor(R * u''^2): low grid cells are visited most;
* with probability 1e-3 the point is invalid: x = NaN or root = -1 (half each), to
  exercise the "no region" answer.

Counters: SplitMix64 of (seed, batch, i, draw) as in :mod:`synth.recipe`; x and y are
rounded once to float32. NumPy only; no arithmetic of the partition itself.
"""

import numpy as np

from .recipe import box_muller, draw, frame_key, mix64, uniform_pair

GAMMA64 = np.uint64(0x9E3779B97F4A7C15)
SPOTS = ((0.3, 0.7), (0.8, 0.2))
SPOT_SD = 0.03


def make_points(n, n_roots, seed, batch=0, chunk=1 << 22):
    """(root int32 [n], x float32 [n], y float32 [n]) for a forest of n_roots trees."""
    root = np.empty(n, dtype=np.int32)
    xs = np.empty(n, dtype=np.float32)
    ys = np.empty(n, dtype=np.float32)
    fk = frame_key(seed, batch)
    for s0 in range(0, n, chunk):
        i = np.arange(s0, min(n, s0 + chunk), dtype=np.uint64)
        with np.errstate(over="ignore"):
            key = mix64(np.uint64(fk) + (i + np.uint64(1)) * GAMMA64)
        u1, u2 = uniform_pair(draw(key, 0))
        u3, u4 = uniform_pair(draw(key, 1))
        u5, u6 = uniform_pair(draw(key, 2))
        u7, u8 = uniform_pair(draw(key, 3))
        z1, z2 = box_muller(u3, u4)
        spot = u5 < 0.5
        second = u6 < 0.5
        cx = np.where(second, SPOTS[1][0], SPOTS[0][0])
        cy = np.where(second, SPOTS[1][1], SPOTS[0][1])
        x = np.where(spot, np.clip(cx + SPOT_SD * z1, 0.0, 1.0), u1 ** 3)
        y = np.where(spot, np.clip(cy + SPOT_SD * z2, 0.0, 1.0), u2)
        r = np.minimum((n_roots * u7 * u7).astype(np.int64), n_roots - 1)
        bad = u8 < 1e-3
        x = np.where(bad & (u6 < 0.5), np.nan, x)
        r = np.where(bad & (u6 >= 0.5), -1, r)
        sl = slice(s0, s0 + len(i))
        root[sl] = r
        xs[sl] = x.astype(np.float32)
        ys[sl] = y.astype(np.float32)
    return root, xs, ys
