"""Seeded stand-in for the direction perturbations an MLT renderer proposes (the paper's
renderer and scenes are not available).

Proposal i of batch b carries the region key of the current state, the current direction
omega (unit) and two uniforms (u, v) that the perturbation turns into theta' and phi':

* key = floor(m u1^2) (low regions visited most), with probability 1e-3 out of range (-1
  or m);
* omega = a normalised standard normal triple (uniform on the sphere), rounded to float32;
  with probability 1e-3 exactly a pole (0, 0, +-1), where the tangent frame switches
  branch;
* (u, v): 24-bit uniforms in [0, 1), exact in float32.

The regions' lambda table: 10 % of the regions at the adaptation's lower limit -30
(sigma = e^-15), 10 % in [3, 6] (sigma up to 20: close to uniform on [-pi, pi]), the rest
uniform in [-8, 3].

Counters: SplitMix64 of (seed, batch, i, draw) as in :mod:`synth.recipe`. NumPy only; no
arithmetic of the perturbation itself.
"""

import numpy as np

from .recipe import box_muller, draw, frame_key, mix64, uniform_pair

GAMMA64 = np.uint64(0x9E3779B97F4A7C15)


def make_lambda_table(m, seed):
    u = np.random.default_rng([seed, 17]).random((m, 2))
    lam = -8.0 + 11.0 * u[:, 1]
    lam = np.where(u[:, 0] < 0.1, -30.0, lam)
    lam = np.where(u[:, 0] > 0.9, 3.0 + 3.0 * u[:, 1], lam)
    return lam


def make_perturb_inputs(n, m, seed, batch=0, chunk=1 << 22):
    """(region int32 [n], omega float32 [n, 3], uv float32 [n, 2])."""
    region = np.empty(n, dtype=np.int32)
    omega = np.empty((n, 3), dtype=np.float32)
    uv = np.empty((n, 2), dtype=np.float32)
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
        z3, _ = box_muller(u5, u6)
        w = np.stack([z1, z2, z3], axis=1)
        w /= np.linalg.norm(w, axis=1, keepdims=True)
        pole = u2 < 1e-3
        w[pole] = 0.0
        w[pole, 2] = np.where(u7[pole] < 0.5, 1.0, -1.0)
        k = np.minimum((m * u1 * u1).astype(np.int64), m - 1)
        bad = u8 < 1e-3
        k = np.where(bad, np.where(u6 < 0.5, -1, m), k)
        u9, u10 = uniform_pair(draw(key, 4))
        sl = slice(s0, s0 + len(i))
        region[sl] = k
        omega[sl] = w.astype(np.float32)
        uv[sl, 0] = u9
        uv[sl, 1] = u10
    return region, omega, uv
