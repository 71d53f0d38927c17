"""Counter-based random numbers and the synthetic scene function (NumPy, vectorised).

Every random quantity is a pure function of integer counters, so the CPU and GPU
generators draw the same numbers without sharing state:

    frame_key(seed, frame)     = mix64(mix64((seed + 1) * GAMMA) + (frame + 1) * GAMMA)
    sample_key(fk, pixel, s)   = mix64(fk + ((pixel << 20) | s) * GAMMA + GAMMA)
    draw(sk, d)                = mix64(sk + (d + 1) * GAMMA)
    uniform_pair(h)            = ((h >> 40) * 2**-24, ((h >> 16) & 0xFFFFFF) * 2**-24)

All arithmetic is modulo 2**64. ``mix64`` is the SplitMix64 output function (Steele, Lea,
Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014) with the
multipliers of Stafford's "Mix13" variant. Sample index ``SAMPLE_PIXEL`` (2**20 - 1) is
reserved for per-pixel draws, so a frame holds at most 2**20 - 2 samples per pixel.
"""

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
SAMPLE_PIXEL = (1 << 20) - 1
MAX_SPP = SAMPLE_PIXEL - 1
_S30 = np.uint64(30)
_S27 = np.uint64(27)
_S31 = np.uint64(31)
_S40 = np.uint64(40)
_S16 = np.uint64(16)
_S20 = np.uint64(20)
_MASK24 = np.uint64(0xFFFFFF)
_INV24 = 1.0 / float(1 << 24)


def _u64(x):
    return np.asarray(x, dtype=np.uint64)


def mix64(z):
    z = _u64(z)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> _S30)) * _M1
        z = (z ^ (z >> _S27)) * _M2
    return z ^ (z >> _S31)


def frame_key(seed, frame):
    with np.errstate(over="ignore"):
        a = mix64((_u64(seed) + np.uint64(1)) * GAMMA)
        return mix64(a + (_u64(frame) + np.uint64(1)) * GAMMA)


def sample_key(fk, pixel, sample):
    with np.errstate(over="ignore"):
        ctr = (_u64(pixel) << _S20) | _u64(sample)
        return mix64(_u64(fk) + ctr * GAMMA + GAMMA)


def draw(sk, d):
    with np.errstate(over="ignore"):
        return mix64(_u64(sk) + (_u64(d) + np.uint64(1)) * GAMMA)


def uniform_pair(h):
    """Two float64 uniforms in [0, 1) with 24 bits each, from one 64-bit hash."""
    h = _u64(h)
    ua = (h >> _S40).astype(np.float64) * _INV24
    ub = ((h >> _S16) & _MASK24).astype(np.float64) * _INV24
    return ua, ub


def box_muller(u1, u2):
    """Two standard normals from two uniforms in [0, 1) (Box and Muller, 1958)."""
    r = np.sqrt(-2.0 * np.log(1.0 - u1))
    t = 2.0 * np.pi * u2
    return r * np.cos(t), r * np.sin(t)


def scene(u, v):
    """Radiance L (3,...), albedo (3,...), normal (3,...), depth (...) at canonical (u, v)."""
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    edge = (u + 0.37 * v) < 0.62
    du = u - 0.7
    dv = v - 0.35
    disc = (du * du + dv * dv) < 0.0225
    att = np.where(edge, 1.0, 0.3)
    L = np.stack([(0.2 + 0.6 * u) * att, (0.2 + 0.6 * v) * att, (0.8 - 0.6 * u) * att])
    disc_rgb = np.array([0.95, 0.85, 0.15]).reshape((3,) + (1,) * u.ndim)
    L = np.where(disc, disc_rgb, L)
    alb = np.where(edge, np.array([0.8, 0.8, 0.8]).reshape(disc_rgb.shape),
                   np.array([0.3, 0.5, 0.7]).reshape(disc_rgb.shape))
    alb = np.where(disc, disc_rgb, alb)
    nx = 0.5 - u
    ny = 0.5 - v
    inv = 1.0 / np.sqrt(nx * nx + ny * ny + 1.0)
    nrm = np.stack([nx * inv, ny * inv, inv])
    nrm = np.where(disc, np.array([0.0, 0.0, 1.0]).reshape(disc_rgb.shape), nrm)
    depth = np.where(disc, 0.5, 1.0 + u)
    return L, alb, nrm, depth
