"""The Python binding refuses caller-supplied output tensors that cannot hold what the
kernels write (wrong shape, dtype, layout or size), before anything is launched."""

import numpy as np
import pytest
import torch

from paper_2402_08273_amd import ops

pytestmark = pytest.mark.gpu


def _f32(*shape):
    return torch.zeros(shape, dtype=torch.float32, device="cuda")


def test_stats_refuses_misshaped_outputs():
    W, H, S = 40, 20, 8
    rad = _f32(3, S, H, W)
    feats = _f32(7, S, H, W)
    good = ops.stats(rad, feats, max_lag=8)
    torch.cuda.synchronize()
    bad_cases = {
        "mean too small": good._replace(mean=_f32(3, H, W - 1)),
        "var float64": good._replace(var=torch.zeros((3, H, W), dtype=torch.float64, device="cuda")),
        "tau not contiguous": good._replace(tau=_f32(3, W, H).transpose(1, 2)),
        "lag_corr with too few lags": good._replace(lag_corr=_f32(3, 4, H, W)),
        "lag_corr plane too small": good._replace(lag_corr=_f32(3, 7, H - 1, W)),
        "feat_mean missing": good._replace(feat_mean=None),
        "feat_var with 3 channels": good._replace(feat_var=_f32(3, H, W)),
    }
    for name, out in bad_cases.items():
        with pytest.raises(ValueError):
            ops.stats(rad, feats, max_lag=8, out=out)
        print("refused:", name, flush=True)
    ops.stats(rad, feats, max_lag=8, out=good)  # the matching set is accepted
    torch.cuda.synchronize()


def test_filter_refuses_misshaped_outputs():
    W, H, N, r, S = 40, 20, 4, 3, 8
    mean = _f32(3, H, W)
    lam = _f32(N * N)
    with pytest.raises(ValueError):
        ops.filter_forward(mean, lam, r, N, out=_f32(3, H, W + 1))
    out = ops.filter_forward(mean, lam, r, N)
    U = _f32(3, H, W)
    for kw in ({"grad_radiance": _f32(3, H - 1, W)},
               {"grad_radiance": torch.zeros((3, H, W), dtype=torch.float16, device="cuda")},
               {"grad_lambda": _f32(N * N - 1)},
               {"grad_lambda": torch.zeros(N * N, dtype=torch.float64, device="cuda")}):
        with pytest.raises(ValueError):
            ops.filter_backward(U, mean, out, lam, r, S, N, **kw)
    with pytest.raises(ValueError):
        ops.filter_backward(_f32(3, H, W - 2), mean, out, lam, r, S, N)
    with pytest.raises(ValueError):
        ops.filter_backward(None, mean, out, lam, r, S, N, reference=_f32(3, H, W),
                            loss=torch.zeros(1, dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        ops.loss_seed(out, _f32(3, H, W), grad_out=_f32(3, H, 2))
    G, gl = ops.filter_backward(U, mean, out, lam, r, S, N)
    torch.cuda.synchronize()
    assert np.all(G.cpu().numpy() == 0) and np.all(gl.cpu().numpy() == 0)


def test_lens_step_refuses_state_on_another_device_or_of_another_type():
    # checked before anything is launched; with no chains nothing would be launched anyway,
    # so a missing check could not reach the kernel with a host pointer
    L = _f32(16, 32)
    lam = torch.zeros(4, dtype=torch.float64, device="cuda")
    om, nz = _f32(0, 3), _f32(0, 3)
    cases = {
        "density on the host": dict(density=torch.zeros(0, dtype=torch.float32)),
        "pixel on the host": dict(pixel=torch.zeros(0, dtype=torch.int32)),
        "pixel int64": dict(pixel=torch.zeros(0, dtype=torch.int64, device="cuda")),
        "pixel of the wrong length": dict(pixel=torch.zeros(3, dtype=torch.int32, device="cuda")),
    }
    for name, kw in cases.items():
        with pytest.raises(ValueError):
            ops.lens_chain_step(L, 0.5, lam, 2, om, nz, **kw)
        print("refused:", name, flush=True)
    with pytest.raises(ValueError):
        ops.lens_chain_step(L, 0.5, lam, 2, torch.zeros((0, 3), dtype=torch.float32), nz)
    region, alpha = ops.lens_chain_step(L, 0.5, lam, 2, om, nz, density=_f32(0),
                                        pixel=torch.zeros(0, dtype=torch.int32, device="cuda"))
    torch.cuda.synchronize()
    assert region.numel() == 0 and alpha.numel() == 0
