"""Full-size parity at 1920 x 1080, 64 spp, 11 x 11 window, 20 x 20 regions, in the launch
configuration the bench times: stats -> filter -> loss seed -> adjoint, each step on the GPU
from the previous GPU step, checked against the FP64 oracle. The oracle runs on the full
frame for the filter, loss and adjoint; per-pixel statistics are checked on row bands that
contain the image border, region boundaries and fireflies."""

import numpy as np
import pytest
import torch

import oracle
from paper_2402_08273_amd import ops
from parity import backward_scales, check, filter_scale, stats_scales
from synth import gpu as sgpu
from synth import make_lambda

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

W, H, S, R, N = 1920, 1080, 64, 5, 20


@pytest.fixture(scope="module")
def frame():
    print("generating 1920x1080x64 frame on the GPU", flush=True)
    rad, feat = sgpu.make_frame(W, H, S, seed=2, frame=0)
    ref = sgpu.make_reference(W, H, seed=1002, frame=0, spp=4096)
    lam = make_lambda(N, seed=99)
    torch.cuda.synchronize()
    return rad, feat, ref, lam


def test_full_frame_chain(frame):
    rad, feat, ref, lam = frame
    lam_d = torch.from_numpy(lam).cuda()
    st = ops.stats(rad, feat, max_lag=8)
    out = ops.filter_forward(st.mean, lam_d, R, N)
    loss, U = ops.loss_seed(out, ref)
    G, gl = ops.filter_backward(U, st.mean, out, lam_d, R, S, N)
    torch.cuda.synchronize()
    print("gpu chain done; oracle on the full frame", flush=True)

    rad_h = rad.cpu().numpy()
    ref_h = ref.cpu().numpy().astype(np.float64)
    mean_o = oracle.stats_accumulate(rad_h, None, 0)["mean"]
    out_o, _ = oracle.filter_forward(mean_o, lam, N, R)
    L_o, U_o = oracle.mse_loss_seed(out_o, ref_h)
    G_o, gl_o = oracle.filter_backward(U_o, mean_o, out_o, lam, N, R, -30.0, S)
    n = out_o.size
    check("out", out.cpu().numpy(), out_o, filter_scale(mean_o, lam, N, R, -30.0))
    u_scale = 2.0 * (np.abs(out_o) + np.abs(ref_h)) / n
    check("U", U.cpu().numpy(), U_o, u_scale)
    d = np.abs(out_o - ref_h)
    check("loss", loss.cpu().numpy()[0], L_o, L_o + (2 * d * (np.abs(out_o) + np.abs(ref_h))).sum() / n)
    G_s, gl_s = backward_scales(u_scale, mean_o, out_o, lam, N, R, -30.0, S)
    check("G", G.cpu().numpy(), G_o, G_s)
    check("grad_lambda", gl.cpu().numpy(), gl_o, gl_s)
    print("oracle chain compared; per-pixel statistics on bands", flush=True)

    feat_h = feat.cpu().numpy()
    for y0, y1 in [(0, 6), (535, 546), (1074, 1080)]:
        sl = slice(y0, y1)
        r_b = rad_h[:, :, sl]
        f_b = feat_h[:, :, sl]
        ref_st = oracle.stats_accumulate(r_b, f_b, 8)
        sc = stats_scales(r_b, ref_st)
        check("mean", st.mean[:, sl].cpu().numpy(), ref_st["mean"], sc["mean"])
        check("var", st.var[:, sl].cpu().numpy(), ref_st["var"], sc["var"])
        check("tau", st.tau[:, sl].cpu().numpy(), ref_st["tau"], sc["tau"])
        check("lag_corr", st.lag_corr[:, :, sl].cpu().numpy(), ref_st["lag_corr"], sc["rho"])
        f64 = f_b.astype(np.float64)
        check("feat_mean", st.feat_mean[:, sl].cpu().numpy(), ref_st["feat_mean"], np.abs(f64).mean(axis=1))
        check("feat_var", st.feat_var[:, sl].cpu().numpy(), ref_st["feat_var"],
              ref_st["feat_var"] + 1e-6 * (f64 * f64).mean(axis=1))
    # the fireflies of this seed are present in the checked bands
    assert (rad_h[:, :, :6] > 10).any()
