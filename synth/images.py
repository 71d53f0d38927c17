"""Seeded image pairs for the rRMSE measure: a reference R and a rendered image I of the
same synthetic scene (the paper's scenes and renders are not available).

R: the scene radiance of :func:`synth.recipe.scene` at the pixel centres, with 1 % of the
pixels black (a black reference pixel is where the eps of the measure matters).
I: R plus per-pixel Gaussian noise of standard deviation uniform in [0.02, 0.5] per pixel,
and with probability 1e-3 per pixel a firefly exp(3 + Z) in all channels -- the error
profile of a noisy render. Both float32 [3][H][W]. NumPy Generator seeded with (seed, W, H);
no arithmetic of the measure itself.
"""

import numpy as np

from .recipe import scene


def make_image_pair(W, H, seed):
    rng = np.random.default_rng([seed, W, H])
    u = (np.arange(W) + 0.5) / W
    v = (np.arange(H) + 0.5) / H
    uu, vv = np.meshgrid(u, v)
    R = scene(uu, vv)[0]
    R = np.where(rng.random((H, W)) < 0.01, 0.0, R)
    sig = rng.uniform(0.02, 0.5, size=(H, W))
    I = R + sig * rng.standard_normal((3, H, W))
    fire = rng.random((H, W)) < 1e-3
    I = I + np.where(fire, np.exp(3.0 + rng.standard_normal((H, W))), 0.0)
    return I.astype(np.float32), R.astype(np.float32)
