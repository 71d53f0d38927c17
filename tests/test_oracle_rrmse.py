"""Pins of the rRMSE oracle (Sec. 8.2 error measure; formula as read in oracle/rrmse.py):
a hand-worked 2x2 image in exact rational arithmetic, zero error for identical images, a
constant relative error, the eps term at black reference pixels, and the consistency of the
map with the image value."""

from fractions import Fraction as Fr

import mpmath
import numpy as np
import pytest

from oracle import rrmse as orr


def test_hand_worked_example():
    # I and R per channel for four pixels; eps = 1/100
    I = np.array([[[1.0, 2.0], [0.0, 0.5]], [[1.0, 1.5], [0.25, 0.5]], [[2.0, 2.0], [0.0, 0.0]]])
    R = np.array([[[1.0, 1.0], [0.5, 0.5]], [[0.5, 1.5], [0.25, 0.0]], [[2.0, 1.0], [0.0, 1.0]]])
    eps = Fr(1, 100)
    e = [[Fr(0)] * 2 for _ in range(2)]
    for y in range(2):
        for x in range(2):
            s = Fr(0)
            for c in range(3):
                i, r = Fr(I[c, y, x]), Fr(R[c, y, x])
                s += (i - r) ** 2 / (r * r + eps)
            e[y][x] = s / 3
    # by hand, pixel (0, 0): (0 + 0.25/0.26 + 0) / 3 = 25/78
    assert e[0][0] == Fr(25, 78)
    m, v = orr.rrmse(I, R, eps=0.01)
    for y in range(2):
        for x in range(2):
            assert m[y, x] == pytest.approx(float(mpmath.sqrt(mpmath.mpf(e[y][x].numerator) / e[y][x].denominator)),
                                            rel=1e-15)
    mean = sum(e[0] + e[1]) / 4
    assert v == pytest.approx(float(mpmath.sqrt(mpmath.mpf(mean.numerator) / mean.denominator)), rel=1e-15)


def test_identical_images_and_constant_relative_error():
    rng = np.random.default_rng(1)
    R = rng.uniform(0.5, 4.0, size=(3, 17, 23))
    m, v = orr.rrmse(R, R)
    assert v == 0.0 and np.all(m == 0.0)
    # I = (1 + d) R: e_j = d^2 mean_c R^2 / (R^2 + eps) -> d^2 as eps -> 0
    d = 0.03
    m, v = orr.rrmse((1 + d) * R, R, eps=0.0)
    assert np.allclose(m, d, rtol=1e-12) and v == pytest.approx(d, rel=1e-12)
    m, v = orr.rrmse((1 + d) * R, R, eps=1e-2)
    assert v < d and v > d * np.sqrt(0.25 / (0.25 + 1e-2)) * 0.999


def test_black_reference_and_consistency():
    R = np.zeros((3, 4, 5))
    I = np.full((3, 4, 5), 0.1)
    m, v = orr.rrmse(I, R, eps=1e-2)
    assert np.allclose(m, 1.0) and v == pytest.approx(1.0)          # 0.01 / (0 + 0.01)
    rng = np.random.default_rng(2)
    I = rng.uniform(0, 3, size=(3, 31, 29))
    R = rng.uniform(0, 3, size=(3, 31, 29))
    m, v = orr.rrmse(I, R)
    assert v == pytest.approx(np.sqrt(np.mean(m ** 2)), rel=1e-14)    # the map squares average to rRMSE^2
