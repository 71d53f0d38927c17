"""GPU parity of rrmse (Sec. 8.2 error measure) against the FP64 oracle. The GPU forms each
pixel's relative squared error in fp64 from the float32 inputs, as the oracle does, and
stores its square root as float32: map within 2^-23 relative. The image value is an fp64
sum in another order: within 1e-12 relative."""

import numpy as np
import pytest
import torch

from oracle import rrmse as orr
from paper_2402_08273_amd import ops
from synth.images import make_image_pair

pytestmark = pytest.mark.gpu


def _check(name, I, R, eps=1e-2):
    m, v = ops.rrmse(torch.from_numpy(I).cuda(), torch.from_numpy(R).cuda(), eps=eps)
    m, v = m.cpu().numpy(), float(v.item())
    wm, wv = orr.rrmse(I, R, eps=eps)
    assert np.array_equal(np.isnan(m), np.isnan(wm)), name
    assert np.array_equal(np.isinf(m), np.isinf(wm)), name
    ok = np.isfinite(wm)
    assert np.all(np.abs(m[ok] - wm[ok]) <= 2.0 ** -23 * wm[ok]), (name, float(np.abs(m[ok] - wm[ok]).max()))
    if not np.isfinite(wv):
        assert (np.isnan(v) and np.isnan(wv)) or v == wv, (name, v, wv)
    else:
        assert abs(v - wv) <= 1e-12 * wv + 1e-300, (name, v, wv)
    return m, v


@pytest.mark.parametrize("W,H", [(1, 1), (97, 61), (1024, 1), (1025, 3), (640, 480)])
def test_rrmse_parity(W, H):
    I, R = make_image_pair(W, H, seed=W + H)
    _check(f"{W}x{H}", I, R)
    _check(f"{W}x{H} eps=0.5", I, R, eps=0.5)


def test_rrmse_edge_cases():
    R = np.zeros((3, 5, 7), dtype=np.float32)
    _, v = _check("zero error", R, R)
    assert v == 0.0
    I = np.full((3, 5, 7), 0.1, dtype=np.float32)
    m, v = _check("black reference", I, R)
    assert np.allclose(m, np.sqrt(np.float64(np.float32(0.1)) ** 2 / 1e-2), rtol=1e-6)
    # eps = 0 at a black pixel with no error: 0/0 -> NaN in the map and the image value
    I2 = I.copy()
    I2[:, 2, 3] = 0.0
    _check("eps 0", I2, R, eps=0.0)
    # only the image value, or only the map
    Id, Rd = torch.from_numpy(I).cuda(), torch.from_numpy(R).cuda()
    m, v = ops.rrmse(Id, Rd, want_map=False)
    assert m is None and float(v) == pytest.approx(orr.rrmse(I, R)[1], rel=1e-12)


def test_rrmse_is_deterministic():
    I, R = make_image_pair(1920, 1080, seed=3)
    Id, Rd = torch.from_numpy(I).cuda(), torch.from_numpy(R).cuda()
    vals = {float(ops.rrmse(Id, Rd)[1].item()) for _ in range(5)}
    assert len(vals) == 1


@pytest.mark.slow
@pytest.mark.parametrize("W,H", [(1920, 1080), (3840, 2160)])
def test_rrmse_full_size(W, H):
    print(f"rrmse full size {W}x{H}", flush=True)
    I, R = make_image_pair(W, H, seed=7)
    _check(f"{W}x{H}", I, R)
