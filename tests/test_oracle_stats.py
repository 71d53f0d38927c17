"""Pins for the oracle's Appendix A statistics (no GPU).

Each test checks the oracle against something other than itself: exact rational
arithmetic on hand-sized sequences, literal loops, closed forms of seeded distributions,
and special cases.
"""

import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from synth import ar1_samples


def _exact_stats(seq, max_lag):
    """Brute force in exact rationals, straight from the definitions."""
    q = [Fraction(v) for v in seq]
    S = len(q)
    mu = sum(q) / S
    M2 = sum((v - mu) ** 2 for v in q)
    var = M2 / (S - 1) if S >= 2 else Fraction(0)
    K = min(max_lag, S - 1)
    C = []
    for k in range(1, K + 1):
        C.append(sum((q[s] - mu) * (q[s + k] - mu) for s in range(S - k)))
    rho = [c / M2 if M2 != 0 else Fraction(0) for c in C]
    tau = 1 + 2 * sum(rho)
    return mu, M2, var, rho, tau


@pytest.mark.parametrize(
    "seq,max_lag",
    [
        ([1, 2, 4, 8], 8),
        ([3.5, -1.25, 0.5], 1),
        ([100.0, 0.5, 0.25, 0.75, 0.5], 8),  # firefly first
        ([2.0], 8),
        ([0.1, 0.2], 0),
        ([1, -1, 1, -1, 1, -1, 1, -1, 1], 4),
    ],
)
def test_exact_rational_sequences(seq, max_lag):
    mu, M2, var, rho, tau = _exact_stats(seq, max_lag)
    st = oracle.chain_statistics(np.array(seq, dtype=np.float64), max_lag)
    assert st["K_L"] == len(rho)
    assert math.isclose(float(st["mu"]), float(mu), rel_tol=1e-15, abs_tol=1e-15)
    assert math.isclose(float(st["M2"]), float(M2), rel_tol=1e-14, abs_tol=1e-14)
    assert math.isclose(float(st["var"]), float(var), rel_tol=1e-14, abs_tol=1e-14)
    for k in range(len(rho)):
        assert math.isclose(float(st["rho"][k]), float(rho[k]), rel_tol=1e-13, abs_tol=1e-14)
    assert math.isclose(float(st["tau"]), float(tau), rel_tol=1e-13, abs_tol=1e-13)


def test_hand_worked_example():
    # g = 1, 2, 4, 8: mean 15/4, deviations -11/4, -7/4, 1/4, 17/4,
    # M2 = (121 + 49 + 1 + 289)/16 = 115/4, var = 115/12,
    # C_1 = (77 - 7 + 17)/16 = 87/16 -> rho_1 = 87/460,
    # C_2 = (-11 + -119)/16 = -130/16 -> rho_2 = -130/460,
    # C_3 = -187/16 -> rho_3 = -187/460; tau = 1 + 2 (87 - 130 - 187)/460 = 1 - 1 = 0.
    st = oracle.chain_statistics(np.array([1.0, 2.0, 4.0, 8.0]), 8)
    assert st["mu"] == 3.75
    assert st["var"] == pytest.approx(115 / 12, rel=1e-15)
    assert st["rho"][:, ...].tolist() == pytest.approx([87 / 460, -130 / 460, -187 / 460], rel=1e-14)
    assert float(st["tau"]) == pytest.approx(0.0, abs=1e-14)


def test_loops_match_vectorised_planes():
    rng = np.random.default_rng(3)
    C, S, H, W = 3, 7, 4, 5
    rad = rng.standard_normal((C, S, H, W)).astype(np.float32)
    rad[0, 0, 1, 1] = 250.0  # firefly
    rad[1, :, 2, 3] = 0.625  # constant pixel
    feats = rng.random((7, S, H, W)).astype(np.float32)
    out = oracle.stats_accumulate(rad, feats, max_lag=8)
    K = min(8, S - 1)
    for c in range(C):
        for y in range(H):
            for x in range(W):
                seq = [float(rad[c, s, y, x]) for s in range(S)]
                mu = math.fsum(seq) / S
                M2 = math.fsum((v - mu) ** 2 for v in seq)
                assert out["mean"][c, y, x] == pytest.approx(mu, rel=1e-14, abs=1e-14)
                assert out["var"][c, y, x] == pytest.approx(M2 / (S - 1), rel=1e-13, abs=1e-14)
                tau = 1.0
                for k in range(1, K + 1):
                    ck = math.fsum((seq[s] - mu) * (seq[s + k] - mu) for s in range(S - k))
                    r = ck / M2 if M2 > 0 else 0.0
                    assert out["lag_corr"][c, k - 1, y, x] == pytest.approx(r, rel=1e-12, abs=1e-13)
                    tau += 2 * r
                assert out["tau"][c, y, x] == pytest.approx(tau, rel=1e-12, abs=1e-12)
    for c in range(7):
        seq = feats[c, :, 2, 2].astype(np.float64)
        assert out["feat_mean"][c, 2, 2] == pytest.approx(seq.mean(), rel=1e-14)
        assert out["feat_var"][c, 2, 2] == pytest.approx(seq.var(ddof=1), rel=1e-12)


def test_constant_pixels_are_exact():
    rad = np.full((3, 9, 2, 3), 0.3, dtype=np.float32)
    out = oracle.stats_accumulate(rad, None, max_lag=8)
    assert np.all(out["mean"] == np.float64(np.float32(0.3)))
    assert np.all(out["var"] == 0.0)
    assert np.all(out["lag_corr"] == 0.0)
    assert np.all(out["tau"] == 1.0)


def test_single_sample_degenerates():
    rad = np.array([5.0, -1.0, 2.0], dtype=np.float32).reshape(3, 1, 1, 1)
    out = oracle.stats_accumulate(rad, None, max_lag=8)
    assert out["K_L"] == 0
    assert out["lag_corr"].shape == (3, 0, 1, 1)
    assert np.all(out["var"] == 0.0)
    assert np.all(out["tau"] == 1.0)
    assert out["mean"].ravel().tolist() == [5.0, -1.0, 2.0]


def test_iid_gaussian_variance_closed_form():
    # iid N(m, s^2): E[var] = s^2; the mean over P pixels has relative standard
    # error sqrt(2 / ((S - 1) P)).
    rng = np.random.default_rng(11)
    S, H, W, s = 16, 64, 64, 0.35
    g = (1.5 + s * rng.standard_normal((1, S, H, W)))
    out = oracle.stats_accumulate(g, None, max_lag=4)
    rel_se = math.sqrt(2.0 / ((S - 1) * H * W))
    assert abs(out["var"].mean() / s**2 - 1.0) < 5 * rel_se
    # iid: every lag correlation averages to about -1/S (bias of the estimator), tau ~ 1
    assert abs(out["lag_corr"].mean()) < 0.1
    assert out["mean"].mean() == pytest.approx(1.5, abs=5 * s / math.sqrt(S * H * W))


@pytest.mark.parametrize("rho", [0.0, 0.5, 0.9])
def test_ar1_autocorrelation_closed_form(rho):
    # AR(1): corr at lag k is rho^k, so the truncated autocorrelation time is
    # 1 + 2 rho (1 - rho^K) / (1 - rho). Estimator bias is O((1 + rho) / S).
    S, K = 2048, 8
    g = ar1_samples(1, S, 16, 16, rho, seed=5)
    out = oracle.stats_accumulate(g, None, max_lag=K)
    for k in range(1, 5):
        tol = 0.005 + 2.0 * k * (1 + rho) / ((1 - rho) * S)
        assert abs(out["lag_corr"][0, k - 1].mean() - rho**k) < tol
    tau_cf = 1.0 + 2.0 * sum(rho**k for k in range(1, K + 1))
    assert abs(out["tau"].mean() - tau_cf) < 0.05 * tau_cf


def test_generator_firefly_moments():
    # Y = exp(3 + Z): E[Y] = e^3.5, E[Y^2] = e^8 (lognormal moments). A generator
    # check for the firefly recipe, using the shared counter-based draws.
    from synth.recipe import box_muller, draw, frame_key, sample_key, uniform_pair

    fk = frame_key(1, 0)
    sk = sample_key(fk, np.arange(400000, dtype=np.uint64), 0)
    u3, u4 = uniform_pair(draw(sk, 2))
    _, z3 = box_muller(u3, u4)
    y = np.exp(3.0 + z3)
    assert y.mean() == pytest.approx(math.exp(3.5), rel=0.03)
    assert np.log(y).std() == pytest.approx(1.0, rel=0.01)
