"""Relative root-mean-square error of an image against a reference (Sec. 8.2, the error
measure of the equal-time comparisons: an error per pixel shown as a map, and one number
for the image), in float64 NumPy.

TEST INFRASTRUCTURE (see the package docstring): only tests/, smoke() and bench.py's
cpu_baseline leg may use it.

The paper names the measure without a formula. Reading: with I and R of shape [3][H][W]
and a small eps in the denominator (so that black reference pixels do not divide by zero;
default 1e-2),

    e_j   = (1/3) sum_c (I_cj - R_cj)^2 / (R_cj^2 + eps)     (relative squared error of pixel j)
    map_j = sqrt(e_j)
    rRMSE = sqrt((1/P) sum_j e_j),  P = H W.
"""

import numpy as np

EPS_DEFAULT = 1e-2


def relative_squared_error(image, reference, eps=EPS_DEFAULT):
    """e_j [H][W] of float32/float64 planes [3][H][W]."""
    image = np.asarray(image, dtype=np.float64)
    reference = np.asarray(reference, dtype=np.float64)
    d = image - reference
    with np.errstate(divide="ignore", invalid="ignore"):  # eps = 0 at a black pixel: inf or NaN
        return np.mean(d * d / (reference * reference + float(eps)), axis=0)


def rrmse(image, reference, eps=EPS_DEFAULT):
    """(map [H][W], image rRMSE)."""
    e = relative_squared_error(image, reference, eps)
    return np.sqrt(e), float(np.sqrt(np.mean(e)))
