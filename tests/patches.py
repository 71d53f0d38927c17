"""Parity of full-size frames on sampled outputs: the oracle recomputes every output of a
patch from the samples of the patch plus a 2r halo (a crop of the frame that keeps the
full frame's regions and border), so frames far too large for a full-frame FP64 oracle
are still checked pixel by pixel, at the sizes and in the launch configuration that the
bench times.

A patch is (x0, y0, w, h) in output pixels. Region patches cover one screen region
exactly, so its dL/dlambda_k is complete and is checked too.
"""

import numpy as np

import oracle
from parity import backward_scales, check, filter_scale, stats_scales


def region_patch(W, H, N, kx, ky):
    """Bounding box (x0, y0, w, h) of region (kx, ky) of a W x H frame."""
    xs = np.nonzero(oracle.region_index(W, 1, N, (0, 0), (1, W))[0] % N == kx)[0]
    ys = np.nonzero(oracle.region_index(1, H, N, (0, 0), (H, 1))[:, 0] // N == ky)[0]
    return int(xs[0]), int(ys[0]), int(xs[-1] - xs[0] + 1), int(ys[-1] - ys[0] + 1)


def _host(t, sl):
    return t[sl].detach().cpu().numpy()


def check_patches(name, gpu, rad, feat, ref, lam, N, R, patches, regions=(), lambda_min=-30.0, max_lag=8):
    """Compare the GPU outputs of one frame with the oracle on every patch and region.

    gpu: dict of device tensors mean, var, tau, out, grad_radiance, grad_lambda, and
    feat_mean, feat_var when feat is given (lag_corr optional); rad [3,S,H,W], feat
    [7,S,H,W] or None, ref [3,H,W]: the device inputs the GPU consumed; lam: host array.
    Returns the number of pixels and regions compared."""
    _, S, H, W = rad.shape
    P = W * H
    todo = [(p, None) for p in patches] + [(region_patch(W, H, N, kx, ky), ky * N + kx) for kx, ky in regions]
    npx = 0
    for (x0, y0, w, h), k in todo:
        assert 0 <= x0 and x0 + w <= W and 0 <= y0 and y0 + h <= H, (x0, y0, w, h)
        cx0, cy0 = max(x0 - 2 * R, 0), max(y0 - 2 * R, 0)
        cx1, cy1 = min(x0 + w + 2 * R, W), min(y0 + h + 2 * R, H)
        csl = (slice(cy0, cy1), slice(cx0, cx1))
        rad_c = _host(rad, (slice(None), slice(None)) + csl)
        feat_c = None if feat is None else _host(feat, (slice(None), slice(None)) + csl)
        ref_c = _host(ref, (slice(None),) + csl).astype(np.float64)
        st = oracle.stats_accumulate(rad_c, feat_c, max_lag)
        crop = dict(origin=(cx0, cy0), image_size=(W, H))
        out_o, _ = oracle.filter_forward(st["mean"], lam, N, R, lambda_min, **crop)
        _, U_o = oracle.mse_loss_seed(out_o, ref_c, count=3 * P)
        G_o, gl_o = oracle.filter_backward(U_o, st["mean"], out_o, lam, N, R, lambda_min, S, **crop)
        # the patch inside the crop, and on the frame
        pc = (slice(None), slice(y0 - cy0, y0 - cy0 + h), slice(x0 - cx0, x0 - cx0 + w))
        pf = (slice(None), slice(y0, y0 + h), slice(x0, x0 + w))
        tag = f"{name} patch ({x0},{y0},{w},{h})"
        sc = stats_scales(rad_c, st)
        check(tag + " mean", _host(gpu["mean"], pf), st["mean"][pc], sc["mean"][pc])
        check(tag + " var", _host(gpu["var"], pf), st["var"][pc], sc["var"][pc])
        check(tag + " tau", _host(gpu["tau"], pf), st["tau"][pc], sc["tau"][pc])
        if gpu.get("lag_corr") is not None:
            lc = (slice(None), slice(None)) + pc[1:]
            check(tag + " lag_corr", _host(gpu["lag_corr"], (slice(None), slice(None)) + pf[1:]),
                  st["lag_corr"][lc], sc["rho"])
        if feat is not None:
            f64 = feat_c.astype(np.float64)
            check(tag + " feat_mean", _host(gpu["feat_mean"], pf), st["feat_mean"][pc],
                  np.abs(f64).mean(axis=1)[pc])
            check(tag + " feat_var", _host(gpu["feat_var"], pf), st["feat_var"][pc],
                  (st["feat_var"] + 1e-6 * (f64 * f64).mean(axis=1))[pc])
        check(tag + " out", _host(gpu["out"], pf), out_o[pc],
              filter_scale(st["mean"], lam, N, R, lambda_min, **crop)[pc])
        u_scale = 2.0 * (np.abs(out_o) + np.abs(ref_c)) / (3 * P)
        G_s, gl_s = backward_scales(u_scale, st["mean"], out_o, lam, N, R, lambda_min, S, **crop)
        check(tag + " G", _host(gpu["grad_radiance"], pf), G_o[pc], G_s[pc])
        if k is not None:
            check(f"{tag} grad_lambda[{k}]", _host(gpu["grad_lambda"], slice(k, k + 1)), gl_o[k:k + 1],
                  gl_s[k:k + 1])
        npx += w * h
    return npx


def check_loss(name, loss, out, ref, tol=1e-6):
    """The fused loss against the FP64 sum over the GPU's own filtered image: checks the
    reduction at full size (out itself is checked on patches)."""
    o = out.detach().cpu().numpy().astype(np.float64)
    r = ref.detach().cpu().numpy().astype(np.float64)
    want = float(((o - r) ** 2).sum() / o.size)
    got = float(loss)
    assert abs(got - want) <= tol * want, (name, got, want)
