"""The 32-frame batch (frames from 256 x 256 to 2048 x 1152, 4 to 256 spp, 11 x 11 window)
in one HIP graph per step: statistics, filter, loss seed and adjoint as one launch each over
the whole batch, in both forms of the step (the loss formed in the forward pass, as the
bench times it, and the seed fused into the adjoint). Every frame is checked against the
oracle on a sampled patch across a region corner and on its four corners (the window
clipped by two frame edges inside the one launch); every fourth frame also on a whole
region (its dL/dlambda_k, with per-frame gradient buffers). The batch loss is checked
against the FP64 sum over the frames' filtered images."""

import numpy as np
import pytest
import torch

from paper_2402_08273_amd.batch import FrameBatch, FrameInput
from patches import check_patches, region_patch
from synth import gpu as sgpu
from synth import make_lambda
from synth.workloads import LAMBDA_SEED, MAX_LAG, N_REGIONS, REFERENCE_SPP, batch32

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.mark.parametrize("loss_in_forward", [True, False], ids=["loss-in-forward", "fused-seed"])
def test_batch32_graph_replay_matches_oracle(loss_in_forward):
    N = N_REGIONS
    lam = make_lambda(N, seed=LAMBDA_SEED)
    lam_d = torch.from_numpy(lam).cuda()
    specs = batch32()
    print("generating 32 frames on the GPU", flush=True)
    frames, inputs = [], []
    for sp in specs:
        rad, feat = sgpu.make_frame(sp.W, sp.H, sp.S, seed=sp.seed, frame=sp.frame)
        ref = sgpu.make_reference(sp.W, sp.H, seed=sp.seed + 1000, frame=sp.frame, spp=REFERENCE_SPP)
        inputs.append((rad, feat, ref))
        frames.append(FrameInput(rad, feat, ref, lam_d, radius=sp.radius, n_regions=N, max_lag=MAX_LAG))
    b = FrameBatch(frames, loss_in_forward=loss_in_forward)
    b.capture()
    b.replay()
    torch.cuda.synchronize()
    print("graph replayed; oracle on sampled patches", flush=True)
    want_loss = 0.0
    for i, (sp, (rad, feat, ref), o) in enumerate(zip(specs, inputs, b.outputs)):
        # a patch across the corner of regions (7, 11) / (8, 12)
        x0, y0, _, _ = region_patch(sp.W, sp.H, N, 8, 12)
        cw, ch = 16, 12
        patches = [(x0 - 12, y0 - 8, 24, 16), (0, 0, cw, ch), (sp.W - cw, 0, cw, ch), (0, sp.H - ch, cw, ch),
                   (sp.W - cw, sp.H - ch, cw, ch)]
        regions = [((3 * i) % N, (7 * i) % N)] if i % 4 == 0 else []
        check_patches(f"frame {i} ({sp.W}x{sp.H}x{sp.S})", o, rad, feat, ref, lam, N, sp.radius, patches, regions)
        d = o["out"].double() - ref.double()
        want_loss += float((d * d).mean())
    got = float(b.loss.cpu()[0])
    assert abs(got - want_loss) <= 1e-6 * want_loss, (got, want_loss)
