"""The GPU generator of the synthetic inputs reproduces the NumPy recipe (the definition).
Transcendentals may differ in the last float64 ulp, so a rare stored value may differ by
one unit in its last place; everything else is bit-identical."""

import numpy as np
import pytest
import torch

from synth import gpu as sgpu
from synth import make_frame, make_reference
from synth.numpy_gen import NOISE_CONST, NOISE_UNIFORM

pytestmark = pytest.mark.gpu


def _ulp_close(a, b, dtype):
    a = np.asarray(a)
    b = np.asarray(b)
    assert a.shape == b.shape
    ia = a.view(np.int32 if dtype == np.float32 else np.int16).astype(np.int64)
    ib = b.view(np.int32 if dtype == np.float32 else np.int16).astype(np.int64)
    diff = np.abs(ia - ib)
    assert diff.max() <= 1, f"max ulp difference {diff.max()}"
    assert (diff > 0).mean() < 1e-4, f"{(diff > 0).sum()} values differ by one ulp"


@pytest.mark.parametrize("noise,fdt", [(NOISE_UNIFORM, np.float32), (NOISE_CONST, np.float16)])
def test_gpu_generator_matches_numpy(noise, fdt):
    W, H, S = 67, 29, 9
    rad, feat = make_frame(W, H, S, seed=5, frame=3, noise=noise, firefly_p=0.05, feature_dtype=fdt)
    tdt = torch.float16 if fdt == np.float16 else torch.float32
    rg, fg = sgpu.make_frame(W, H, S, seed=5, frame=3, noise=noise, firefly_p=0.05, feature_dtype=tdt)
    torch.cuda.synchronize()
    _ulp_close(rg.cpu().numpy(), rad, np.float32)
    _ulp_close(fg.cpu().numpy(), feat, fdt)


def test_gpu_reference_matches_numpy():
    W, H = 31, 17
    ref = make_reference(W, H, seed=1001, spp=40)
    rg = sgpu.make_reference(W, H, seed=1001, spp=40)
    torch.cuda.synchronize()
    _ulp_close(rg.cpu().numpy(), ref, np.float32)
