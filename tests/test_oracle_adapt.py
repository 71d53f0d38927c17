"""Pins of the regional adaptation oracle (Algorithm 1; eqs. est_exp_acc, update_lambda,
step_size_n; parameters of Sec. 8.1)."""

import math

import numpy as np
import pytest

from oracle import region_adapt as ra


def _run(m, region, alpha, **kw):
    return ra.adapt(ra.initial_state(m), region, alpha, **kw)


def test_hand_worked_example():
    # m = 2, L = 2, alpha* = 0.5, gamma_max = 1, gamma_scale = 5 (worked by hand):
    # region 0: (0.25, 0.5) -> mean 0.375 < 0.5 -> lambda 1 - min(1, 5/1) = 0, n = 2
    #           (1.0, 1.0)  -> mean 1 > 0.5    -> lambda 0 + min(1, 5/sqrt 2) = 1, n = 3
    # region 1: (0.5, 0.5)  -> mean = target   -> sgn 0, lambda stays 1, n = 2
    #           (0.75)      -> one visit pending: A = 0.75, i = 1
    region = [0, 1, 0, 1, 0, 0, 1]
    alpha = [0.25, 0.5, 0.5, 0.5, 1.0, 1.0, 0.75]
    st = _run(2, region, alpha, L=2)
    assert st["lambda"].tolist() == [1.0, 1.0]
    assert st["updates"].tolist() == [3, 2]
    assert st["visits"].tolist() == [0, 1]
    assert st["acc"].tolist() == [0.0, 0.75]
    # stop region 0 after its first window: lambda 0
    st = _run(2, region[:3], alpha[:3], L=2)
    assert st["lambda"].tolist() == [0.0, 1.0]


def test_step_size_schedule():
    # Sec. 8.1: gamma_max = 1, gamma_scale = 5, so gamma_n = 1 up to n = 25, then 5 / sqrt n
    assert [ra.step_size(n) for n in (1, 4, 25)] == [1.0, 1.0, 1.0]
    assert ra.step_size(26) < 1.0 and ra.step_size(100) == 0.5
    assert ra.step_size(10 ** 6) == pytest.approx(5e-3)


def test_constant_acceptance_above_target_follows_the_step_sum():
    # alpha = 0.75 every visit: every window mean is exactly 0.75 > 0.5, so lambda grows by
    # gamma_n at update n. For J > 25 updates the sum lies within the integral bounds of
    # sum_{n=26}^{J} 5 / sqrt(n): [10 (sqrt(J+1) - sqrt 26), 10 (sqrt J - sqrt 25)].
    L, J = 10, 400
    st = _run(1, np.zeros(L * J, np.int64), np.full(L * J, 0.75, np.float32), L=L)
    grow = st["lambda"][0] - 1.0
    lo = 25 + 10 * (math.sqrt(J + 1) - math.sqrt(26))
    hi = 25 + 10 * (math.sqrt(J) - math.sqrt(25))
    assert lo <= grow <= hi
    assert st["updates"][0] == J + 1 and st["visits"][0] == 0


def test_constant_acceptance_below_target_stops_at_lambda_min():
    L = 10
    st = _run(1, np.zeros(L * 30, np.int64), np.full(L * 30, 0.125, np.float32), L=L)
    # 25 unit steps down from 1, then 5/sqrt(26) ~ 0.98 ... : 30 updates stay above -30
    assert -30.0 < st["lambda"][0] < -24.0
    st = _run(1, np.zeros(L * 200, np.int64), np.full(L * 200, 0.125, np.float32), L=L)
    assert st["lambda"][0] == -30.0  # clamped, and stays there


def test_estimator_is_the_regional_mean_and_the_decomposition_holds():
    # With L beyond the stream length no update fires: A_k / i_k is eq. est_exp_acc, the
    # mean acceptance of the visits to region k; and the overall mean minus the target is
    # sum_k b_k (alpha_hat_k - alpha*) with b_k = M_k / M, sum_k b_k = 1 (Sec. 5.3).
    rng = np.random.default_rng(4)
    m, n = 7, 5000
    region = rng.integers(0, m, n)
    alpha = rng.random(n).astype(np.float32)
    st = _run(m, region, alpha, L=10 ** 9)
    counts = np.bincount(region, minlength=m)
    means = np.bincount(region, weights=alpha.astype(np.float64), minlength=m) / counts
    assert np.array_equal(st["visits"], counts)
    np.testing.assert_allclose(st["acc"] / st["visits"], means, rtol=1e-13)
    b = counts / n
    assert b.sum() == pytest.approx(1.0)
    astar = 0.5
    assert alpha.astype(np.float64).mean() - astar == pytest.approx(np.sum(b * (means - astar)), abs=1e-12)
    assert np.all(st["lambda"] == 1.0) and np.all(st["updates"] == 1)


def test_batches_compose_and_regions_are_independent():
    rng = np.random.default_rng(5)
    m, n = 12, 4000
    region = rng.integers(-1, m + 1, n)  # a few out-of-range entries: skipped
    alpha = rng.random(n).astype(np.float32)
    whole = _run(m, region, alpha, L=7)
    # two batches with the state carried over
    st = ra.initial_state(m)
    ra.adapt(st, region[:1234], alpha[:1234], L=7)
    ra.adapt(st, region[1234:], alpha[1234:], L=7)
    for key in whole:
        assert np.array_equal(whole[key], st[key]), key
    # any interleaving that keeps each region's own order gives the same state
    perm = np.argsort(rng.permutation(m + 2)[region + 1], kind="stable")
    shuffled = _run(m, region[perm], alpha[perm], L=7)
    for key in whole:
        assert np.array_equal(whole[key], shuffled[key]), key
    # conservation: every valid visit is either in a completed window or pending
    valid = ((region >= 0) & (region < m)).sum()
    assert ((whole["updates"] - 1) * 7 + whole["visits"]).sum() == valid
    assert np.all(whole["visits"] < 7) and np.all(whole["lambda"] >= -30.0)


def test_update_direction_follows_the_equation():
    # eq. update_lambda: acceptance above the target increases lambda, below decreases it
    up = _run(1, [0] * 10, [0.9] * 10)
    down = _run(1, [0] * 10, [0.1] * 10)
    assert up["lambda"][0] == 2.0 and down["lambda"][0] == 0.0
