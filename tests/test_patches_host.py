"""The sampled-output parity machinery (tests/patches.py) on the CPU: outputs computed by
the full-frame oracle pass every patch and region check, and a planted error in any of
them is caught."""

import numpy as np
import pytest
import torch

import oracle
from patches import check_loss, check_patches, region_patch
from synth import make_frame, make_lambda, make_reference

W, H, S, R, N = 90, 64, 12, 3, 5  # S > max_lag + 1: tau = 1 + 2 sum rho is 0 when K_L = S - 1


@pytest.fixture(scope="module")
def frame():
    rad, feat = make_frame(W, H, S, seed=5, feature_dtype=np.float16)
    ref = make_reference(W, H, seed=1005, spp=16)
    lam = make_lambda(N, seed=99)
    st = oracle.stats_accumulate(rad, feat, 8)
    out, _ = oracle.filter_forward(st["mean"], lam, N, R)
    L, U = oracle.mse_loss_seed(out, ref)
    G, gl = oracle.filter_backward(U, st["mean"], out, lam, N, R, -30.0, S)
    outputs = {k: torch.from_numpy(np.ascontiguousarray(v)) for k, v in
               dict(mean=st["mean"], var=st["var"], tau=st["tau"], lag_corr=st["lag_corr"],
                    feat_mean=st["feat_mean"], feat_var=st["feat_var"], out=out, grad_radiance=G,
                    grad_lambda=gl).items()}
    return (torch.from_numpy(rad), torch.from_numpy(feat), torch.from_numpy(ref), lam, outputs, L)


PATCHES = [(0, 0, 10, 8), (30, 20, 25, 20), (80, 50, 10, 14)]
REGIONS = [(0, 0), (2, 3), (4, 4)]


def test_region_patches_tile_the_frame():
    area = 0
    for ky in range(N):
        for kx in range(N):
            x0, y0, w, h = region_patch(W, H, N, kx, ky)
            k = oracle.region_index(W, H, N)[y0:y0 + h, x0:x0 + w]
            assert (k == ky * N + kx).all()
            area += w * h
    assert area == W * H


def test_oracle_outputs_pass(frame):
    rad, feat, ref, lam, outputs, L = frame
    n = check_patches("oracle", outputs, rad, feat, ref, lam, N, R, PATCHES, REGIONS)
    assert n == sum(w * h for _, _, w, h in PATCHES) + sum(
        region_patch(W, H, N, kx, ky)[2] * region_patch(W, H, N, kx, ky)[3] for kx, ky in REGIONS)
    check_loss("oracle", L, outputs["out"], ref)


@pytest.mark.parametrize("key,index", [("mean", (1, 3, 5)), ("tau", (0, 25, 40)), ("out", (2, 0, 0)),
                                       ("grad_radiance", (0, 22, 31)), ("grad_lambda", (2 * N + 3,)),
                                       ("feat_var", (6, 60, 82)), ("lag_corr", (0, 0, 4, 4))])
def test_planted_errors_are_caught(frame, key, index):
    rad, feat, ref, lam, outputs, _ = frame
    bad = dict(outputs)
    bad[key] = outputs[key].clone()
    # 1 % of the value plus 1 % of the tensor's largest magnitude (values can be ~0)
    bad[key][index] += 1e-2 * (abs(float(bad[key][index])) + float(outputs[key].abs().max()))
    regions = REGIONS + [(3, 2)]
    with pytest.raises(AssertionError):
        check_patches("planted", bad, rad, feat, ref, lam, N, R, PATCHES + [(20, 20, 20, 10)], regions)
