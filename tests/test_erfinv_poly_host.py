"""The inverse-error-function polynomials of the perturbation kernel
(paper_2402_08273_amd/csrc/erfinv_poly.hpp), evaluated on the CPU in fp64 exactly as the
kernel composes them (w = -log(x (2 - x)) from the complement x, with the kernel's own
logarithm from the atanh series, Horner in the normalised variable, y times the
polynomial), against mpmath's erfinv at 80 digits: relative error below 1e-9 over every
piece, its ends, and the smallest complement a float32 u gives. The logarithm is also
checked on its own against mpmath's over (0, 1].

The kernel stores theta' = sigma sqrt 2 erfinv(y) as float32: with erfinv's relative error
eps, |theta_f32 - theta| <= 2^-24 |theta| (rounding) + eps |theta| (1 + 2^-24), within the
2^-23 relative bound of the GPU parity tests for eps < 2^-24 ~ 6e-8."""

import math
import os
import re

import mpmath as mp
import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "paper_2402_08273_amd", "csrc", "erfinv_poly.hpp")
BOUND = 1e-9


def _pieces():
    text = open(HEADER).read()
    out = {}
    for name in ("Central", "Tail1", "Tail2", "Tail3"):
        get = lambda key: float(re.search(rf"k{name}{key} = ([^;]+);", text).group(1))  # noqa: E731
        coeffs = re.search(rf"k{name}\[\d+\] = \{{([^}}]+)\}};", text).group(1)
        out[name] = dict(lo=get("Lo"), hi=get("Hi"), scale=get("Scale"), shift=get("Shift"),
                         c=[float(v) for v in coeffs.split(",")])
    return out


PIECES = _pieces()


def _horner(c, t):
    p = c[0]
    for ck in c[1:]:
        p = p * t + ck   # fp64; the kernel fuses each step (fma), a difference of <= 1 ulp per step
    return p


SQRT_HALF = 0.70710678118654752440
LN2 = 0.69314718055994530942


def log_unit(v):
    """The kernel's logarithm of v in [0, 1] (log_unit in perturb.hip), step by step in fp64:
    v = m 2^e, m in [sqrt(1/2), sqrt(2)), e ln 2 + 2 f (1 + f^2/3 + ... + f^14/15),
    f = (m - 1) / (m + 1) (the kernel fuses the multiply-adds: <= 1 ulp per step apart)."""
    if v == 0.0:
        return -math.inf
    m, e = math.frexp(v)
    if m < SQRT_HALF:
        m, e = m + m, e - 1
    f = (m - 1.0) / (m + 1.0)
    f2 = f * f
    p = 1.0 / 15.0
    for c in (1.0 / 13.0, 1.0 / 11.0, 1.0 / 9.0, 1.0 / 7.0, 1.0 / 5.0, 1.0 / 3.0, 1.0):
        p = p * f2 + c
    return e * LN2 + 2.0 * f * p


def test_log_unit_against_mpmath():
    # relative error of the series logarithm over (0, 1]: near 1 (no cancellation, e = 0), at
    # and around powers of two and sqrt(1/2) (the ends of the mantissa range), random
    # points, and the smallest arguments the kernel can form (x (2 - x) >= 2^-147)
    rng = np.random.default_rng(5)
    vs = [1.0, 1.0 - 2.0 ** -53, 1.0 - 1e-12, 1.0 - 1e-6, 0.999, 0.75, 0.5, 0.5 + 2.0 ** -53, 0.5 - 2.0 ** -54,
          SQRT_HALF, math.nextafter(SQRT_HALF, 0.0), math.nextafter(SQRT_HALF, 1.0), 2.0 ** -147, 2.0 ** -1022,
          2.0 ** -1074, 1e-300, 1e-30, 3e-8]
    vs += list(rng.random(2000)) + list(2.0 ** -rng.uniform(0, 140, 2000))
    worst = 0.0
    with mp.workdps(40):
        for v in vs:
            want = mp.log(mp.mpf(v))
            got = log_unit(v)
            rel = abs((mp.mpf(got) - want) / want) if want != 0 else abs(mp.mpf(got))
            worst = max(worst, float(rel))
    assert worst < 2e-13, worst
    assert log_unit(0.0) == -math.inf and math.isnan(log_unit(math.nan))


def erfinv_kernel(y, x):
    """The kernel's composition, in fp64 (None where the kernel defers to erfcinv)."""
    w = -log_unit(x * (2.0 - x))
    c = PIECES["Central"]
    if w < c["hi"]:
        return y * _horner(c["c"], w * c["scale"] + c["shift"])
    s = math.sqrt(w)
    for name in ("Tail1", "Tail2", "Tail3"):
        p = PIECES[name]
        if s < p["hi"] or (name == "Tail3" and s <= p["hi"]):
            return y * _horner(p["c"], s * p["scale"] + p["shift"])
    return None


def _exact(y, x):
    """erfinv of the argument at 80 digits, from whichever of y and its complement x
    determines it: y in the central piece, x in the tails (where y rounds towards 1 and
    erfinv is ill-conditioned in y)."""
    with mp.workdps(80):
        if -math.log(x * (2.0 - x)) < PIECES["Central"]["hi"]:
            return mp.erfinv(mp.mpf(y))
        return mp.erfinv(1 - mp.mpf(x))


def _check(y, x):
    got = erfinv_kernel(y, x)
    assert got is not None, (y, x)
    want = _exact(y, x)
    rel = abs((mp.mpf(got) - want) / want) if want != 0 else abs(mp.mpf(got))
    assert rel < BOUND, (y, x, got, float(want), float(rel))
    return float(rel)


def test_header_pieces_tile_the_range():
    c, t1, t2, t3 = (PIECES[n] for n in ("Central", "Tail1", "Tail2", "Tail3"))
    assert c["lo"] == 0.0 and t1["lo"] == math.sqrt(c["hi"]) and t1["hi"] == t2["lo"] and t2["hi"] == t3["lo"]
    # the smallest complement of a float32 u in (0, 1): 2 * 2^-149 (e <= 1), or 2^-149 with e >= 1/2
    assert math.sqrt(-math.log(2.0 ** -149 * 2.0)) < t3["hi"]
    # w = 0 gives erfinv'(0) = sqrt(pi) / 2
    assert abs(_horner(c["c"], -1.0) - math.sqrt(math.pi) / 2) < 1e-10


@pytest.mark.parametrize("name", ["Central", "Tail1", "Tail2", "Tail3"])
def test_relative_error_over_each_piece(name):
    p = PIECES[name]
    worst = 0.0
    for v in np.linspace(p["lo"], p["hi"], 301):
        w = v if name == "Central" else v * v
        if w == 0.0:
            continue
        # y and its complement x, each from w to full relative precision (as the kernel has them)
        q = math.exp(-w)
        y = math.sqrt(-math.expm1(-w))
        x = q / (1.0 + math.sqrt(1.0 - q))
        if name != "Central" and -math.log(x * (2.0 - x)) < PIECES["Central"]["hi"]:
            continue  # the rounding of w sends the first tail point to the central piece
        worst = max(worst, _check(y, x))
    assert worst < BOUND


def test_small_and_float32_edge_arguments():
    # y tiny (w rounds to 0): erfinv(y) = y sqrt(pi) / 2 to first order
    for y in [1e-300, 2.0 ** -40, 2.0 ** -20, 1e-3]:
        _check(y, 1.0 - y)
    # complements from float32 u near 0 with e = 1 (sigma small): x = 2u
    for u in [2.0 ** -149, 2.0 ** -126, 1e-30, 2.0 ** -24, 1e-7, 3e-4, 0.01, 0.3]:
        x = 2.0 * u
        _check(1.0 - x, x)
