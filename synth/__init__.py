"""Seeded synthetic render buffers shared by the tests, the bench and the oracle checks.

This module produces *inputs only*: Monte Carlo radiance sample planes, feature sample
planes, a high-spp reference image and a per-region parameter table. It contains none
of the arithmetic of the statistics/filter path itself. Two implementations of one
recipe exist:

* :mod:`synth.numpy_gen` -- plain NumPy, for small frames on the CPU;
* :mod:`synth.gpu` -- a HIP kernel (``synth/csrc/synth.hip``) for large frames, checked
  against the NumPy version in the GPU tests.

Recipe (stands in for the paper's scenes, which are not available; the paper renders
with path-space MLT and splats contributions to the film, Sec. 3.1):

* counter-based random numbers: SplitMix64 finaliser (Steele, Lea, Flood 2014) applied to
  ``(seed, frame, pixel, sample, draw)`` counters, 24-bit uniforms, Box-Muller Gaussians;
* jittered sample position ``u = (x + xi_x)/W``, ``v = (y + xi_y)/H``;
* scene: linear colour ramp, one straight hard edge (attenuation 0.3), one flat disc;
* noise: ``g = L + sigma_p * Z`` per channel, ``sigma_p`` constant or uniform in
  [0.02, 0.5] per pixel;
* fireflies: with probability ``firefly_p`` per sample, ``exp(3 + Z)`` added to all
  three channels (lognormal(3, 1));
* features: albedo (3), normal (3), depth (1) evaluated at the jittered position;
* everything is evaluated in float64 and rounded once to the storage type.
"""

from .recipe import (  # noqa: F401
    GAMMA,
    SAMPLE_PIXEL,
    mix64,
    frame_key,
    sample_key,
    draw,
    uniform_pair,
)
from .numpy_gen import (  # noqa: F401
    make_frame,
    make_reference,
    make_lambda,
    ar1_samples,
)
