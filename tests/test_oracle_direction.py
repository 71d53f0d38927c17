"""Pins of the direction-perturbation oracle (Sec. 3.3 "Perturbing Ray Directions", the scale
sigma = sqrt(exp(lambda)) of Sec. 5.3): the inverse CDF against the plain definition at 60
digits, a Kolmogorov-Smirnov test and the inverse identity against the exact CDF, the
closed-form moments of the truncated normal, its small- and large-sigma limits, and the
geometry of the Duff et al. (2017) frame and of the proposed direction."""

import math

import mpmath
import numpy as np
import pytest
from scipy import special

from oracle import direction_sampler as ds

SIGMAS = [1e-6, 1e-3, 0.1, 0.7, 1.0, 3.0, 30.0, 1e4, 1e9]


def _plain(u, sigma):
    """theta' = sigma Phi^-1(Phi(-a) + u (Phi(a) - Phi(-a))), with 60 significant digits."""
    with mpmath.workdps(60):
        s = mpmath.mpf(sigma)
        a = mpmath.pi / s
        lo, hi = mpmath.ncdf(-a), mpmath.ncdf(a)
        p = lo + mpmath.mpf(u) * (hi - lo)
        if p <= 0:
            return -math.pi
        if p >= 1:
            return math.pi
        return float(s * mpmath.sqrt(2) * mpmath.erfinv(2 * p - 1))


@pytest.mark.parametrize("sigma", SIGMAS)
def test_inverse_cdf_matches_the_plain_definition(sigma):
    us = [0.0, 1e-300, 1e-12, 1e-7, 1e-3, 0.25, 0.4999, 0.5, 0.5001, 0.75, 0.999, 1 - 1e-7, 1 - 2.0 ** -24]
    got = ds.truncated_normal_theta(np.array(us), sigma)
    for u, g in zip(us, got):
        want = _plain(u, sigma)
        assert abs(g - want) <= 1e-13 * abs(want) + 1e-50 * sigma, (sigma, u, g, want)  # 60-digit rounding
        assert -math.pi <= g <= math.pi


@pytest.mark.parametrize("sigma", [0.05, 1.0, 2.5, 40.0])
def test_kolmogorov_smirnov_against_the_exact_cdf(sigma):
    n = 200_000
    u = np.random.default_rng(7).random(n)
    theta = ds.truncated_normal_theta(u, sigma)
    F = ds.truncated_normal_cdf(theta, sigma)     # through ndtr, not erfinv
    # the inverse identity F(theta(u)) = u
    assert np.max(np.abs(F - u)) < 1e-12
    Fs = np.sort(F)
    i = np.arange(1, n + 1)
    D = max(np.max(i / n - Fs), np.max(Fs - (i - 1) / n))
    assert D < 1.95 / math.sqrt(n)               # 0.1 % critical value


@pytest.mark.parametrize("sigma", [0.02, 0.5, 1.0, 2.0, 6.0])
def test_moments_of_the_truncated_normal(sigma):
    # midpoint rule over u of E[g(theta)], against the closed forms of the normal
    # truncated to [-a, a] in units of sigma (a = pi / sigma)
    N = 1 << 21
    u = (np.arange(N) + 0.5) / N
    th = ds.truncated_normal_theta(u, sigma)
    a = math.pi / sigma
    Z = special.ndtr(a) - special.ndtr(-a)
    pdf = lambda z: math.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)
    assert abs(th.mean()) < 1e-12
    assert np.allclose(th, -th[::-1], rtol=0, atol=1e-13)            # theta(1 - u) = -theta(u)
    var = sigma ** 2 * (1 - 2 * a * pdf(a) / Z)
    mabs = 2 * sigma * (pdf(0) - pdf(a)) / Z
    assert abs(np.mean(th * th) - var) < 2e-5 * var
    assert abs(np.mean(np.abs(th)) - mabs) < 2e-5 * mabs


def test_limits():
    # small sigma: the normal quantile (z_0.975 = 1.959963984540054, textbook value)
    s = 1e-3
    assert ds.truncated_normal_theta(0.975, s) / s == pytest.approx(1.959963984540054, rel=1e-12)
    assert ds.truncated_normal_theta(0.5, s) == 0.0
    # large sigma: uniform on [-pi, pi]
    u = np.linspace(0, 1, 101)
    assert np.allclose(ds.truncated_normal_theta(u, 1e6), (2 * u - 1) * np.pi, atol=1e-9)
    # the ends of the support
    assert ds.truncated_normal_theta(0.0, 1e-6) == -math.pi
    assert ds.truncated_normal_theta(1.0, 0.3) == pytest.approx(math.pi, abs=1e-12)


def test_frame_is_orthonormal_and_right_handed():
    rng = np.random.default_rng(3)
    n = rng.normal(size=(2000, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    n = np.concatenate([n, [[0, 0, 1], [0, 0, -1], [0, 0, -0.0], [1, 0, 0], [0, -1, 0]]])
    n[-3] = [1e-9, 0, -1]
    n[-3] /= np.linalg.norm(n[-3])
    t, b = ds.frame(n)
    dot = lambda p, q: np.sum(p * q, axis=1)
    assert np.allclose(dot(t, n), 0, atol=1e-14) and np.allclose(dot(b, n), 0, atol=1e-14)
    assert np.allclose(dot(t, b), 0, atol=1e-14)
    assert np.allclose(dot(t, t), 1, atol=1e-14) and np.allclose(dot(b, b), 1, atol=1e-14)
    assert np.allclose(np.cross(t, b), n, atol=1e-14)
    # the poles, by hand from the published formulas
    t0, b0 = ds.frame(np.array([[0.0, 0.0, 1.0], [0.0, 0.0, -1.0]]))
    assert t0.tolist() == [[1.0, 0.0, 0.0], [1.0, 0.0, 0.0]]
    assert b0.tolist() == [[0.0, 1.0, 0.0], [0.0, -1.0, 0.0]]


def test_proposed_direction_geometry():
    rng = np.random.default_rng(4)
    m, n = 5, 5000
    lam = np.array([-30.0, -4.0, 0.0, 1.0, 6.0])
    region = rng.integers(-1, m + 1, n)
    w = rng.normal(size=(n, 3))
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    uv = rng.random((n, 2))
    uv[:10, 0] = 0.5
    out, theta = ds.perturb_directions(lam, region, w, uv)
    ok = (region >= 0) & (region < m)
    assert np.all(np.isnan(out[~ok])) and np.all(np.isnan(theta[~ok]))
    o, w_, th, uv_ = out[ok], w[ok], theta[ok], uv[ok]
    assert np.allclose(np.sum(o * o, axis=1), 1, atol=1e-14)
    assert np.allclose(np.sum(o * w_, axis=1), np.cos(th), atol=1e-14)        # the polar angle
    t, b = ds.frame(w_)
    phi = 2 * np.pi * uv_[:, 1]
    assert np.allclose(np.sum(o * t, axis=1), np.sin(th) * np.cos(phi), atol=1e-14)
    assert np.allclose(np.sum(o * b, axis=1), np.sin(th) * np.sin(phi), atol=1e-14)
    # u = 1/2: no perturbation; sigma from lambda
    mid = ok.copy()
    mid[10:] = False
    assert np.allclose(out[mid], w[mid], atol=1e-15)
    assert ds.sigma_of(1.0) == pytest.approx(math.exp(0.5), rel=1e-15)
    # lambda = -30 (the clamp of the adaptation): sigma = e^-15, angles of that order
    small = ok & (region == 0)
    assert np.all(np.abs(theta[small]) < 20 * math.exp(-15))
