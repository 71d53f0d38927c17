"""Regional adaptation of the scaling parameters lambda_k from a stream of proposals
(Algorithm 1 of the paper, with eqs. est_exp_acc, update_lambda and step_size_n), in
float64, one proposal at a time in stream order.

TEST INFRASTRUCTURE (see the package docstring): only tests/, smoke() and bench.py's
cpu_baseline leg may use it.

Each proposal i carries the region k_i of the current state (Alg. 1, line 8) and its
acceptance probability alpha_i = alpha(x_i, y_i) (line 11). Per region the algorithm keeps
lambda_k (initial scaling parameter, Sec. 8.1: 1), the visit count i_k, the accumulated
acceptance A_k and the update count n_k (initially 1), and for every visit:

    A_k += alpha_i;  i_k += 1
    once i_k reaches L:  alpha_hat = A_k / L                      (eq. est_exp_acc)
                         gamma     = min(gamma_max, gamma_scale n_k^(-1/2))   (eq. step_size_n)
                         lambda_k  = lambda_k + gamma sgn(alpha_hat - alpha*) (eq. update_lambda)
                         i_k = A_k = 0;  n_k += 1

Readings where the paper is inconsistent or silent:

* the listing triggers when i_k exceeds L but divides by L; the update here fires when i_k
  reaches L, so alpha_hat is the mean of exactly the L accumulated visits;
* the prose of Sec. 5.3 states the direction of the update the other way round from eq.
  update_lambda; the equation is followed (lambda grows when the estimated acceptance is
  above the target);
* lambda is limited below by the minimum scaling parameter (Sec. 8.1, -30) after every
  update: lambda_k = max(lambda_k + gamma sgn(...), lambda_min);
* sgn(0) = 0;
* regions are independent (Sec. 5.3, "Criterion for Adaptation"), and within a region the
  proposals are taken in stream order; a proposal whose region is outside [0, m) is
  skipped;
* alpha_i arrives as a float32 value and is accumulated in float64.
"""

import math

import numpy as np

L_DEFAULT = 10
GAMMA_MAX_DEFAULT = 1.0
GAMMA_SCALE_DEFAULT = 5.0
ALPHA_TARGET_DEFAULT = 0.5
LAMBDA_INIT_DEFAULT = 1.0
LAMBDA_MIN_DEFAULT = -30.0


def initial_state(m, lambda_init=LAMBDA_INIT_DEFAULT):
    """Alg. 1 lines 2-7 for m regions: lambda, A (float64), i, n (int64)."""
    return {
        "lambda": np.full(m, float(lambda_init), dtype=np.float64),
        "acc": np.zeros(m, dtype=np.float64),
        "visits": np.zeros(m, dtype=np.int64),
        "updates": np.ones(m, dtype=np.int64),
    }


def step_size(n, gamma_max=GAMMA_MAX_DEFAULT, gamma_scale=GAMMA_SCALE_DEFAULT):
    """eq. step_size_n: gamma_n = min(gamma_max, gamma_scale / sqrt(n))."""
    return min(gamma_max, gamma_scale / math.sqrt(n))


def adapt(state, region, alpha, L=L_DEFAULT, gamma_max=GAMMA_MAX_DEFAULT, gamma_scale=GAMMA_SCALE_DEFAULT,
          alpha_target=ALPHA_TARGET_DEFAULT, lambda_min=LAMBDA_MIN_DEFAULT):
    """Run the proposals (region[i], alpha[i]) through Algorithm 1's adaptation in stream
    order, updating ``state`` (from :func:`initial_state`) in place; returns it."""
    lam, acc, vis, upd = state["lambda"], state["acc"], state["visits"], state["updates"]
    m = lam.shape[0]
    region = np.asarray(region).astype(np.int64)
    alpha = np.asarray(alpha, dtype=np.float32).astype(np.float64)
    for k, a in zip(region.tolist(), alpha.tolist()):
        if k < 0 or k >= m:
            continue
        acc[k] += a
        vis[k] += 1
        if vis[k] >= L:
            alpha_hat = float(acc[k]) / L
            gamma = step_size(int(upd[k]), gamma_max, gamma_scale)
            sgn = int(alpha_hat > alpha_target) - int(alpha_hat < alpha_target)
            lam[k] = max(float(lam[k]) + gamma * sgn, lambda_min)
            vis[k] = 0
            acc[k] = 0.0
            upd[k] += 1
    return state
