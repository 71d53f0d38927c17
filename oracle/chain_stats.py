"""Appendix A statistics of each pixel's Monte Carlo sample sequence, in float64.

TEST INFRASTRUCTURE (see the package docstring): only tests/, smoke() and bench.py's
cpu_baseline leg may use it.

The paper's Appendix A ("Correlation and Convergence") writes the MCMC estimator of a pixel
as the mean of g(x_i) = f(x_i) / (pi(x_i)/b) (also Sec. 3.2, the estimator of I_j), its
asymptotic variance as var(g) + 2 sum_k cov(g(x_1), g(x_{1+k})), the autocorrelation time
tau = 1 + 2 sum_k corr(g(x_1), g(x_{1+k})) with corr := cov / var, and the effective sample
size N_eff = N / tau.

Readings applied here (the paper states these for a chain, not for a buffer of samples):

* the sequence of a pixel is its samples in buffer order s = 0 .. S-1;
* mean  mu = (1/S) sum_s g_s;  M2 = sum_s (g_s - mu)^2 (two passes);
  var = M2 / (S - 1) for S >= 2, else 0;
* lag autocovariance sums C_k = sum_{s=0}^{S-1-k} (g_s - mu)(g_{s+k} - mu);
  rho_k = C_k / M2 (the 1/S of the covariance and of the variance cancel);
* the infinite sum of tau is truncated at K_L = min(max_lag, S - 1): tau = 1 + 2 sum rho_k;
  tau is not clamped;
* a sequence with M2 = 0 (all samples equal) has rho_k = 0 and tau = 1.
"""

import numpy as np


def pixel_moments(g):
    """Mean, M2 and sample variance of sequences along the last axis.

    g: float array [..., S]. Returns (mu, M2, var) as float64 arrays [...].
    """
    g = np.asarray(g, dtype=np.float64)
    S = g.shape[-1]
    mu = g.sum(axis=-1) / S
    dev = g - mu[..., None]
    M2 = (dev * dev).sum(axis=-1)
    if S >= 2:
        var = M2 / (S - 1)
    else:
        var = np.zeros_like(M2)
    return mu, M2, var


def lag_autocovariances(g, mu, K_L):
    """C_k for k = 1..K_L along the last axis. Returns float64 [K_L, ...]."""
    g = np.asarray(g, dtype=np.float64)
    S = g.shape[-1]
    dev = g - mu[..., None]
    out = np.zeros((K_L,) + g.shape[:-1])
    for k in range(1, K_L + 1):
        out[k - 1] = (dev[..., : S - k] * dev[..., k:]).sum(axis=-1)
    return out


def chain_statistics(g, max_lag=8):
    """All Appendix A statistics of sequences along the last axis.

    Returns dict with mu, M2, var, rho [K_L, ...], tau, K_L.
    """
    g = np.asarray(g, dtype=np.float64)
    S = g.shape[-1]
    K_L = min(int(max_lag), S - 1)
    mu, M2, var = pixel_moments(g)
    C = lag_autocovariances(g, mu, K_L)
    positive = M2 > 0.0
    safe = np.where(positive, M2, 1.0)
    rho = np.where(positive[None], C / safe[None], 0.0)
    tau = 1.0 + 2.0 * rho.sum(axis=0)
    return {"mu": mu, "M2": M2, "var": var, "rho": rho, "tau": tau, "K_L": K_L}


def stats_accumulate(radiance, features=None, max_lag=8):
    """Per-pixel statistics of sample planes laid out [c][s][y][x].

    radiance: [3, S, H, W]; features: [7, S, H, W] or None.
    Returns dict: mean, var, tau [3,H,W]; lag_corr [3,K_L,H,W]; M2 [3,H,W];
    feat_mean, feat_var [7,H,W] (if features given). All float64.
    """
    rad = np.moveaxis(np.asarray(radiance, dtype=np.float64), 1, -1)  # [3,H,W,S]
    st = chain_statistics(rad, max_lag)
    out = {
        "mean": st["mu"],
        "var": st["var"],
        "tau": st["tau"],
        "M2": st["M2"],
        "lag_corr": np.moveaxis(st["rho"], 0, 1),  # [3,K_L,H,W]
        "K_L": st["K_L"],
    }
    if features is not None:
        f = np.moveaxis(np.asarray(features, dtype=np.float64), 1, -1)
        fm, _, fv = pixel_moments(f)
        out["feat_mean"] = fm
        out["feat_var"] = fv
    return out
