"""Full-size parity at 3840 x 2160, 256 spp, FP16-stored features, 15 x 15 window, in the
launch configuration the bench times (statistics without the lag planes, filter, fused
loss seed + adjoint). The oracle recomputes sampled outputs from crops of the frame:
image corners and edges, a 2 x 2 region corner, and five whole regions (their
dL/dlambda_k is complete)."""

import numpy as np
import pytest
import torch

from paper_2402_08273_amd import ops
from patches import check_loss, check_patches
from synth import gpu as sgpu
from synth import make_lambda
from synth.workloads import LAMBDA_SEED, MAX_LAG, N_REGIONS, REFERENCE_SPP, UHD

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def test_uhd_fp16_features_forward_backward():
    W, H, S, R, N = UHD.W, UHD.H, UHD.S, UHD.radius, N_REGIONS
    print(f"generating {W}x{H}x{S} frame (fp16 features) on the GPU", flush=True)
    rad, feat = sgpu.make_frame(W, H, S, seed=UHD.seed, frame=UHD.frame, feature_dtype=torch.float16)
    ref = sgpu.make_reference(W, H, seed=UHD.seed + 1000, frame=UHD.frame, spp=REFERENCE_SPP)
    lam = make_lambda(N, seed=LAMBDA_SEED)
    lam_d = torch.from_numpy(lam).cuda()
    st = ops.stats(rad, feat, MAX_LAG, with_lag_corr=False)
    out = ops.filter_forward(st.mean, lam_d, R, N)
    loss = torch.zeros(1, device="cuda", dtype=torch.float64)
    G, gl = ops.filter_backward(None, st.mean, out, lam_d, R, S, N, reference=ref, loss=loss)
    torch.cuda.synchronize()
    print("gpu chain done; oracle on sampled patches", flush=True)
    gpu = dict(mean=st.mean, var=st.var, tau=st.tau, feat_mean=st.feat_mean, feat_var=st.feat_var, out=out,
               grad_radiance=G, grad_lambda=gl)
    patches = [(0, 0, 48, 24), (1900, 1066, 40, 28), (3792, 2136, 48, 24), (3820, 1000, 20, 30),
               (0, 2140, 30, 20), (180, 100, 24, 16)]
    regions = [(0, 0), (10, 10), (19, 19), (19, 0), (4, 13)]
    n = check_patches("uhd", gpu, rad, feat, ref, lam, N, R, patches, regions)
    print(f"{n} pixels compared", flush=True)
    check_loss("uhd", loss.cpu().numpy()[0], out, ref)
    # fireflies (lognormal(3, 1) on top of L <= 0.95) are inside the checked patches
    assert (rad[:, :, :24, :48] > 10).any()
