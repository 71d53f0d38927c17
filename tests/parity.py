"""Scaled-error parity checks between the HIP path and the FP64 oracle.

A quantity passes iff |gpu - oracle| <= TOL * scale elementwise, with the scale computed
by the oracle in float64 from the magnitudes that enter each computation (so that a
quantity whose true value is ~0, such as a lag correlation or a gradient, is judged
against the size of the terms it is built from). For positive, well-conditioned
quantities this is plain relative error.

Scales (mean over samples written mean_s):
  mean       mean_s |g|
  var        var + 1e-6 mean_s g^2
  rho_k      1
  tau        1 + 2 sum_k |rho_k|
  out        filter(|mean|)                  (same weights, absolute values)
  U          2 (|out| + |R|) / (3P)          (magnitudes entering out - R)
  G          (1/S) sum_j U*_j h_jp / D_j     with U* the U scale (or |U| for given U)
  dL/dlam_k  sum_{j in k} sum_c U*_jc sum_p h'_jp (|mean_p| + |out_j|) / D_j
  loss       L + sum 2 |out - R| (|out| + |R|) / (3P)
"""

import numpy as np

import oracle

TOL = 1e-5


def check(name, gpu, ref, scale, tol=TOL, mask=None):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.broadcast_to(np.asarray(scale, dtype=np.float64), ref.shape)
    err = np.abs(gpu - ref)
    bad = ~(err <= tol * scale)
    if mask is not None:
        bad &= np.broadcast_to(mask, bad.shape)
    if np.any(bad):
        idx = np.argwhere(bad)[:5]
        worst = np.nanmax(np.where(bad, err / np.maximum(scale, 1e-300), 0))
        details = [(tuple(i), float(gpu[tuple(i)]), float(ref[tuple(i)]), float(scale[tuple(i)])) for i in idx]
        raise AssertionError(f"{name}: {int(bad.sum())} of {bad.size} exceed {tol} x scale "
                             f"(worst ratio {worst:.3g}); first (index, gpu, oracle, scale): {details}")
    return float(np.max(err / np.maximum(scale, 1e-300))) if err.size else 0.0


def stats_scales(radiance, st):
    """Scales for mean/var/rho/tau from float samples [3,S,H,W] and oracle stats."""
    g = np.asarray(radiance, dtype=np.float64)
    mean_abs = np.abs(g).mean(axis=1)
    mean_sq = (g * g).mean(axis=1)
    return {
        "mean": mean_abs,
        "var": st["var"] + 1e-6 * mean_sq,
        "rho": 1.0,
        "tau": 1.0 + 2.0 * np.abs(st["lag_corr"]).sum(axis=1),
    }


def filter_scale(mean, lam, n_regions, radius, lambda_min, **crop):
    out, _ = oracle.filter_forward(np.abs(mean), lam, n_regions, radius, lambda_min, **crop)
    return out


def backward_scales(u_scale, mean, out, lam, n_regions, radius, lambda_min, S, **crop):
    """Scales for G and dL/dlambda given a non-negative per-pixel U scale (``crop``:
    origin / image_size as for the oracle)."""
    G_s, gl_s = oracle.filter_backward(u_scale, np.abs(mean), -np.abs(out), lam, n_regions, radius,
                                       lambda_min, S, **crop)
    return G_s, gl_s
