"""Seeded stand-in for the stream of proposals an MLT renderer feeds to the regional
adaptation (the paper's renderer and scenes are not available).

Proposal i of batch b carries a region key and an acceptance probability:

* key_i = floor(m * u1^2): a skewed visit distribution (low keys visited most, like the
  bright image regions a Markov chain dwells in);
* alpha_i = min(1, exp(s_k Z)) with Z standard normal and s_k = 0.25 + 2.5 (k mod 7) / 7:
  the acceptance probability of a symmetric random-walk proposal whose log target ratio
  is normal with a spread that depends on the region, so some regions accept above and
  some below a target of 0.5, and about half the proposals are accepted outright;
* with probability 1e-3 the key is out of range (-1 or m), to exercise skipping.

Counters: SplitMix64 of (seed, batch, i, draw) as in :mod:`synth.recipe`; alpha is rounded
once to float32. NumPy only; no arithmetic of the adaptation itself.
"""

import numpy as np

from .recipe import box_muller, draw, frame_key, mix64, uniform_pair

GAMMA64 = np.uint64(0x9E3779B97F4A7C15)


def make_proposals(n, m, seed, batch=0, chunk=1 << 22):
    """(region int32 [n], alpha float32 [n]) for m regions."""
    region = np.empty(n, dtype=np.int32)
    alpha = np.empty(n, dtype=np.float32)
    fk = frame_key(seed, batch)
    for s0 in range(0, n, chunk):
        i = np.arange(s0, min(n, s0 + chunk), dtype=np.uint64)
        with np.errstate(over="ignore"):
            key = mix64(np.uint64(fk) + (i + np.uint64(1)) * GAMMA64)
        u1, u2 = uniform_pair(draw(key, 0))
        u3, u4 = uniform_pair(draw(key, 1))
        k = np.minimum((m * u1 * u1).astype(np.int64), m - 1)
        z, _ = box_muller(u3, u4)
        s = 0.25 + 2.5 * (k % 7) / 7.0
        a = np.minimum(1.0, np.exp(s * z))
        _, u5 = uniform_pair(draw(key, 2))
        bad = u5 < 1e-3
        k = np.where(bad, np.where(u2 < 0.5, -1, m), k)
        region[s0:s0 + len(i)] = k
        alpha[s0:s0 + len(i)] = a.astype(np.float32)
    return region, alpha
