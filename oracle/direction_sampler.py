"""Perturbation of a ray direction (Sec. 3.3 "Perturbing Ray Directions", with the scale
parameterisation of Sec. 5.3), in float64 NumPy.

TEST INFRASTRUCTURE (see the package docstring): only tests/, smoke() and bench.py's
cpu_baseline leg may use it.

Around the current direction omega, the proposal takes the polar angle theta' from the
normal distribution N(0, sigma^2) truncated to [-pi, pi] and the azimuth phi' uniformly
from [0, 2 pi); sigma_k = sqrt(exp(lambda_k)) is the scale of the region k of the current
state (lambda = log sigma^2). With uniforms (u, v) in [0, 1):

    theta' = sigma Phi^-1(Phi(-a) + u (Phi(a) - Phi(-a))),  a = pi / sigma     (inverse CDF)
    phi'   = 2 pi v
    omega' = sin(theta') cos(phi') t + sin(theta') sin(phi') b + cos(theta') omega

(Phi the standard normal CDF). (t, b, omega) is the orthonormal basis of Duff, Burgess,
Christensen, Hery, Kensler, Liani, Villemin, "Building an Orthonormal Basis, Revisited"
(JCGT 6(1), 2017): the paper leaves the frame's azimuth origin open (any choice gives the
same distribution), and this one fixes it for element-wise comparisons.

Evaluation of the inverse CDF: with e = erf(a / sqrt 2), 2p - 1 = (2u - 1) e and
Phi^-1(p) = sqrt 2 erfinv(2p - 1). For |2p - 1| < 1/2 that is evaluated as written; above,
as sign(2u - 1) sqrt 2 erfcinv(x) with x = 1 - |2p - 1| = 2 min(u, 1 - u) e + erfc(a / sqrt 2)
formed from the complements, so that theta' keeps its relative precision at both ends and
for every sigma (the plain formula loses it where p is close to 0, 1 or 1/2). A result
outside [-pi, pi] (only at u = 0, where Phi(-a) underflows) is clamped to the support.
The plain formula, evaluated with 60 significant digits, pins this evaluation.
"""

import math

import numpy as np
from scipy import special

SQRT2 = math.sqrt(2.0)


def sigma_of(lam):
    """sigma = sqrt(exp(lambda)) (Sec. 5.3)."""
    return np.sqrt(np.exp(np.asarray(lam, dtype=np.float64)))


def truncated_normal_theta(u, sigma):
    """theta' for uniforms u in [0, 1] and scales sigma > 0 (arrays broadcast)."""
    u = np.asarray(u, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    # sigma = 0 or inf (lambda = -inf or +inf) give 0 * inf = NaN where the limit is undefined
    with np.errstate(divide="ignore", over="ignore", invalid="ignore"):
        a = np.pi / sigma
        e = special.erf(a / SQRT2)
        ec = special.erfc(a / SQRT2)
        y = np.abs(2.0 * u - 1.0) * e                   # |2p - 1|
        x = 2.0 * np.minimum(u, 1.0 - u) * e + ec      # 1 - |2p - 1|
        z = np.where(y < 0.5, SQRT2 * special.erfinv(y), SQRT2 * special.erfcinv(x))
        theta = np.sign(u - 0.5) * sigma * z
    return np.clip(theta, -np.pi, np.pi)


def truncated_normal_cdf(theta, sigma):
    """F(theta) = (Phi(theta / sigma) - Phi(-a)) / (Phi(a) - Phi(-a)) on [-pi, pi]."""
    theta = np.asarray(theta, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    a = np.pi / sigma
    return (special.ndtr(theta / sigma) - special.ndtr(-a)) / (special.ndtr(a) - special.ndtr(-a))


def frame(n):
    """Duff et al. 2017 basis (t, b) of unit vectors n [..., 3]: t x b = n."""
    n = np.asarray(n, dtype=np.float64)
    x, y, z = n[..., 0], n[..., 1], n[..., 2]
    s = np.copysign(1.0, z)
    a = -1.0 / (s + z)
    b = x * y * a
    t = np.stack([1.0 + s * x * x * a, s * b, -s * x], axis=-1)
    bb = np.stack([b, s + y * y * a, -y], axis=-1)
    return t, bb


def perturb_directions(lam, region, omega, uv):
    """Proposed directions for proposals i: region[i] (key into lam, the regions' lambda),
    omega[i] (unit, [n, 3]), uv[i] = (u, v). Returns (omega' [n, 3], theta' [n]); a region
    outside [0, len(lam)) gives NaN."""
    lam = np.asarray(lam, dtype=np.float64)
    region = np.asarray(region).astype(np.int64)
    omega = np.asarray(omega, dtype=np.float64)
    uv = np.asarray(uv, dtype=np.float64)
    ok = (region >= 0) & (region < lam.shape[0])
    sigma = np.where(ok, sigma_of(lam[np.where(ok, region, 0)]), np.nan)
    theta = truncated_normal_theta(uv[:, 0], sigma)
    phi = 2.0 * np.pi * uv[:, 1]
    t, b = frame(omega)
    st = np.sin(theta)
    out = (st * np.cos(phi))[:, None] * t + (st * np.sin(phi))[:, None] * b + np.cos(theta)[:, None] * omega
    return out, theta
