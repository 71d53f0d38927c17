"""GPU parity of every hot-path step against the FP64 oracle, on small seeded inputs that
span several tiles and ragged tails. All calls go through the C ABI (via the ctypes
binding); inputs are produced on the CPU (synth / oracle), never by the HIP path."""

import numpy as np
import pytest
import torch

import oracle
from paper_2402_08273_amd import _abi, ops
from parity import TOL, backward_scales, check, filter_scale, stats_scales
from synth import ar1_samples, make_frame, make_lambda, make_reference
from synth.numpy_gen import NOISE_CONST, NOISE_UNIFORM

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _check_stats(rad, feats, max_lag, st_gpu, feat_dtype=np.float32):
    ref = oracle.stats_accumulate(rad, feats, max_lag)
    sc = stats_scales(rad, ref)
    check("mean", _host(st_gpu.mean), ref["mean"], sc["mean"])
    check("var", _host(st_gpu.var), ref["var"], sc["var"])
    check("tau", _host(st_gpu.tau), ref["tau"], sc["tau"])
    if st_gpu.lag_corr is not None:
        lc = _host(st_gpu.lag_corr)
        assert lc.shape == ref["lag_corr"].shape
        check("lag_corr", lc, ref["lag_corr"], sc["rho"])
    if feats is not None:
        f64 = feats.astype(np.float64)
        check("feat_mean", _host(st_gpu.feat_mean), ref["feat_mean"], np.abs(f64).mean(axis=1))
        check("feat_var", _host(st_gpu.feat_var), ref["feat_var"],
              ref["feat_var"] + 1e-6 * (f64 * f64).mean(axis=1))


@pytest.mark.parametrize(
    "W,H,S,max_lag",
    [
        (37, 23, 1, 8), (37, 23, 2, 8), (37, 23, 3, 8), (64, 4, 4, 8), (33, 17, 16, 8),
        (300, 7, 17, 8), (129, 65, 33, 8), (61, 5, 64, 8), (17, 9, 100, 8),
        (40, 6, 20, 0), (40, 6, 20, 1), (40, 6, 20, 3), (23, 11, 70, 32), (23, 11, 40, 16),
    ],
)
def test_stats_parity(W, H, S, max_lag):
    print(f"stats parity W={W} H={H} S={S} max_lag={max_lag}", flush=True)
    rad, feats = make_frame(W, H, S, seed=1 + W + S, noise=NOISE_UNIFORM, firefly_p=0.02)
    # firefly as the first sample of a few pixels, and constant pixels
    rad[:, 0, 0, : min(W, 5)] = 400.0
    rad[:, :, H - 1, W - 1] = 0.625
    st = ops.stats(_dev(rad), _dev(feats), max_lag=max_lag)
    _check_stats(rad, feats, max_lag, st)


@pytest.mark.parametrize("rho", [0.5, 0.9, -0.6])
def test_stats_parity_correlated_sequences(rho):
    # AR(1) sequences give lag correlations far from zero.
    rad = ar1_samples(3, 96, 13, 70, rho, seed=3) * np.float32(0.2) + np.float32(0.5)
    st = ops.stats(_dev(rad), None, max_lag=8)
    _check_stats(rad, None, 8, st)


def test_stats_parity_fp16_features_and_strided_layout():
    W, H, S = 45, 19, 24
    rad, feats = make_frame(W, H, S, seed=4, feature_dtype=np.float16)
    # sample-major allocation with padded rows: [S][C][H][Wpad] viewed as [C][S][H][W]
    Wp = 53
    big = torch.zeros((S, 3, H, Wp), dtype=torch.float32, device="cuda")
    big[:, :, :, :W] = _dev(np.transpose(rad, (1, 0, 2, 3)))
    rad_view = big.permute(1, 0, 2, 3)[:, :, :, :W]
    fbig = torch.zeros((S, 7, H, Wp), dtype=torch.float16, device="cuda")
    fbig[:, :, :, :W] = _dev(np.transpose(feats, (1, 0, 2, 3)))
    f_view = fbig.permute(1, 0, 2, 3)[:, :, :, :W]
    st = ops.stats(rad_view, f_view, max_lag=8)
    _check_stats(rad, feats, 8, st)


def test_stats_without_lag_output_and_features():
    rad, _ = make_frame(19, 7, 9, seed=8, with_features=False)
    st = ops.stats(_dev(rad), None, max_lag=8, with_lag_corr=False)
    assert st.lag_corr is None and st.feat_mean is None
    _check_stats(rad, None, 8, st)


def test_stats_launch_sizes_give_the_same_results():
    # the frame's tiles run as a series of launches of v workgroups per compute unit (or one
    # launch): 1172 tiles, the last one ragged; every launch size gives the same bits, and the
    # default matches the oracle
    W, H, S = 1000, 300, 8
    print(f"stats launch sizes W={W} H={H} S={S}", flush=True)
    rad, feats = make_frame(W, H, S, seed=21, noise=NOISE_UNIFORM, firefly_p=0.01)
    rad_d, feat_d = _dev(rad), _dev(feats)
    results = {}
    for v in (0, 1, 2, 3, 5, _abi.RAMLT_STATS_ONE_LAUNCH):
        f, out = ops.stats_frame(rad_d, feat_d, 4)
        f.flags = v << _abi.RAMLT_STATS_WG_SHIFT
        _abi.stats_accumulate([f], stream=torch.cuda.current_stream().cuda_stream)
        results[v] = [_host(t) for t in out]
    for v, arrs in results.items():
        for name, a, b in zip(ops.Stats._fields, arrs, results[0]):
            assert np.array_equal(a, b, equal_nan=True), (v, name)
    _check_stats(rad, feats, 4, ops.Stats(*[torch.from_numpy(a) for a in results[0]]))


def _filter_inputs(W, H, S, N, seed):
    rad, _ = make_frame(W, H, S, seed=seed, with_features=False)
    mean32 = oracle.stats_accumulate(rad, None, 0)["mean"].astype(np.float32)
    lam = make_lambda(N, seed=99)
    return rad, mean32, lam


@pytest.mark.parametrize(
    "W,H,N,r",
    [
        (70, 37, 3, 3), (128, 128, 20, 3), (41, 9, 5, 5), (100, 50, 7, 7), (33, 20, 20, 15),
        (5, 3, 2, 6), (1, 1, 1, 2), (67, 31, 1, 0), (96, 54, 40, 5), (200, 3, 4, 1),
    ],
)
def test_filter_forward_parity(W, H, N, r):
    print(f"forward parity W={W} H={H} N={N} r={r}", flush=True)
    _, mean32, lam = _filter_inputs(W, H, 4, N, seed=W * 7 + H)
    lam[:: max(1, N)] = -35.0  # some regions below the clamp
    out = ops.filter_forward(_dev(mean32), _dev(lam), r, N, -30.0)
    ref, _ = oracle.filter_forward(mean32, lam, N, r, -30.0)
    check("out", _host(out), ref, filter_scale(mean32, lam, N, r, -30.0))


SCHEDULES = [_abi.RAMLT_TILE_32X16, _abi.RAMLT_TILE_64X8, _abi.RAMLT_TILE_32X8 | _abi.RAMLT_SCHED_DIRECT,
             _abi.RAMLT_TILE_64X8 | _abi.RAMLT_SCHED_DIRECT]


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("W,H,N,r", [(130, 70, 4, 3), (96, 54, 40, 5), (333, 190, 3, 7), (41, 9, 5, 15)])
def test_filter_schedules_parity(W, H, N, r, schedule):
    # every tile shape and the direct gather: forward and adjoint against the oracle
    print(f"schedule {schedule} W={W} H={H} N={N} r={r}", flush=True)
    _, mean32, lam = _filter_inputs(W, H, 4, N, seed=W * 3 + H)
    lam[:: max(1, N)] = -35.0
    out = ops.filter_forward(_dev(mean32), _dev(lam), r, N, -30.0, schedule=schedule)
    ref, _ = oracle.filter_forward(mean32, lam, N, r, -30.0)
    check("out", _host(out), ref, filter_scale(mean32, lam, N, r, -30.0))
    out32 = ref.astype(np.float32)
    S = 8
    U32 = (np.random.default_rng(W).standard_normal((3, H, W)) * 1e-3).astype(np.float32)
    G, gl = ops.filter_backward(_dev(U32), _dev(mean32), _dev(out32), _dev(lam), r, S, N, schedule=schedule)
    G_ref, gl_ref = oracle.filter_backward(U32, mean32, out32, lam, N, r, -30.0, S)
    G_s, gl_s = backward_scales(np.abs(U32), mean32, out32, lam, N, r, -30.0, S)
    check("G", _host(G), G_ref, G_s)
    check("grad_lambda", _host(gl), gl_ref, gl_s)


def test_filter_forward_invariants_on_gpu():
    W, H, N, r = 77, 41, 6, 5
    lam = make_lambda(N, seed=5)
    const = np.full((3, H, W), 0.3125, dtype=np.float32)
    out = _host(ops.filter_forward(_dev(const), _dev(lam), r, N))
    np.testing.assert_allclose(out, 0.3125, rtol=2e-6)
    ident = np.random.default_rng(1).random((3, H, W)).astype(np.float32)
    out = _host(ops.filter_forward(_dev(ident), _dev(np.full(N * N, -30.0, np.float32)), r, N))
    assert np.array_equal(out, ident)


def test_loss_seed_parity():
    W, H = 53, 29
    rng = np.random.default_rng(3)
    out32 = rng.random((3, H, W)).astype(np.float32)
    ref32 = rng.random((3, H, W)).astype(np.float32)
    loss, U = ops.loss_seed(_dev(out32), _dev(ref32))
    L_ref, U_ref = oracle.mse_loss_seed(out32, ref32)
    n = out32.size
    u_scale = 2.0 * (np.abs(out32) + np.abs(ref32)) / n
    check("U", _host(U), U_ref, u_scale)
    d = np.abs(out32.astype(np.float64) - ref32)
    check("loss", _host(loss)[0], L_ref, L_ref + (2 * d * (np.abs(out32) + np.abs(ref32))).sum() / n)


@pytest.mark.parametrize(
    "W,H,N,r,S",
    [
        (70, 37, 3, 3, 16), (41, 9, 5, 5, 4), (33, 20, 20, 15, 1), (5, 3, 2, 6, 3),
        (96, 54, 4, 5, 64), (128, 128, 20, 3, 16), (67, 31, 1, 0, 2),
    ],
)
def test_filter_backward_parity(W, H, N, r, S):
    print(f"backward parity W={W} H={H} N={N} r={r} S={S}", flush=True)
    _, mean32, lam = _filter_inputs(W, H, 4, N, seed=W + 11 * H)
    lam[1 % (N * N)] = -31.0
    out32 = oracle.filter_forward(mean32, lam, N, r)[0].astype(np.float32)
    U32 = (np.random.default_rng(W).standard_normal((3, H, W)) * 1e-3).astype(np.float32)
    G, gl = ops.filter_backward(_dev(U32), _dev(mean32), _dev(out32), _dev(lam), r, S, N)
    G_ref, gl_ref = oracle.filter_backward(U32, mean32, out32, lam, N, r, -30.0, S)
    G_s, gl_s = backward_scales(np.abs(U32), mean32, out32, lam, N, r, -30.0, S)
    check("G", _host(G), G_ref, G_s)
    check("grad_lambda", _host(gl), gl_ref, gl_s)
    assert _host(gl)[1 % (N * N)] == 0.0 or N == 1


def test_chain_parity_small_frame():
    # 128 x 128, 16 spp, 7 x 7 window: stats -> filter -> loss seed -> adjoint, each step
    # on the GPU from the previous GPU step, against the oracle end to end.
    W, H, S, N, r = 128, 128, 16, 20, 3
    rad, feats = make_frame(W, H, S, seed=1, noise=NOISE_CONST, sigma=0.1)
    ref = make_reference(W, H, seed=1001, spp=64, noise=NOISE_CONST, sigma=0.1)
    lam = make_lambda(N, seed=99)
    st = ops.stats(_dev(rad), _dev(feats), max_lag=8)
    out = ops.filter_forward(st.mean, _dev(lam), r, N)
    loss, U = ops.loss_seed(out, _dev(ref))
    G, gl = ops.filter_backward(U, st.mean, out, _dev(lam), r, S, N)

    o = oracle.stats_accumulate(rad, feats, 8)
    out_o, _ = oracle.filter_forward(o["mean"], lam, N, r)
    L_o, U_o = oracle.mse_loss_seed(out_o, ref)
    G_o, gl_o = oracle.filter_backward(U_o, o["mean"], out_o, lam, N, r, -30.0, S)

    _check_stats(rad, feats, 8, st)
    check("out", _host(out), out_o, filter_scale(o["mean"], lam, N, r, -30.0))
    n = out_o.size
    u_scale = 2.0 * (np.abs(out_o) + np.abs(ref)) / n
    check("U", _host(U), U_o, u_scale)
    d = np.abs(out_o - ref)
    check("loss", _host(loss)[0], L_o, L_o + (2 * d * (np.abs(out_o) + np.abs(ref))).sum() / n)
    G_s, gl_s = backward_scales(u_scale, o["mean"], out_o, lam, N, r, -30.0, S)
    check("G", _host(G), G_o, G_s)
    check("grad_lambda", _host(gl), gl_o, gl_s)


@pytest.mark.parametrize("schedule", [0, _abi.RAMLT_TILE_32X8 | _abi.RAMLT_SCHED_DIRECT])
@pytest.mark.parametrize("W,H,N,r", [(96, 54, 4, 5), (70, 37, 20, 3)])
def test_filter_nan_and_infinite_lambda(W, H, N, r, schedule):
    # A NaN lambda propagates as the oracle's exp(max(lambda, lambda_min)) propagates it: out
    # of that region, G within r of it, its dL/dlambda and the loss are NaN, the rest is as
    # for finite lambda; lambda = +inf is a box filter (sigma^2 = inf), -inf is clamped.
    print(f"nan lambda W={W} H={H} N={N} r={r} schedule={schedule}", flush=True)
    _, mean32, lam = _filter_inputs(W, H, 4, N, seed=W + H)
    lam[[1, N + 2]] = np.nan
    lam[N * N - 1] = np.inf
    lam[N] = -np.inf
    out = _host(ops.filter_forward(_dev(mean32), _dev(lam), r, N, -30.0, schedule=schedule))
    ref, _ = oracle.filter_forward(mean32, lam, N, r, -30.0)
    assert np.array_equal(np.isnan(out), np.isnan(ref)) and np.isnan(ref).any()
    ok = ~np.isnan(ref)
    check("out", np.where(ok, out, 0), np.where(ok, ref, 0), np.nan_to_num(filter_scale(mean32, lam, N, r, -30.0)))
    out32 = ref.astype(np.float32)
    S = 4
    U32 = (np.random.default_rng(W).standard_normal((3, H, W)) * 1e-3).astype(np.float32)
    G, gl = (_host(t) for t in ops.filter_backward(_dev(U32), _dev(mean32), _dev(out32), _dev(lam), r, S, N,
                                                   schedule=schedule))
    G_ref, gl_ref = oracle.filter_backward(U32, mean32, out32, lam, N, r, -30.0, S)
    G_s, gl_s = backward_scales(np.abs(U32), mean32, out32, lam, N, r, -30.0, S)
    for name, a, b, s in (("G", G, G_ref, G_s), ("grad_lambda", gl, gl_ref, gl_s)):
        nan = np.isnan(b)
        assert np.array_equal(np.isnan(a), nan), name
        assert nan.any() and not nan.all(), name
        check(name, np.where(nan, 0, a), np.where(nan, 0, b), np.nan_to_num(s))
    # the fused seed: U = 2 (out - R) / (3P) is NaN where out is
    R32 = (mean32 + np.float32(0.01)).astype(np.float32)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    G2, gl2 = (_host(t) for t in ops.filter_backward(None, _dev(mean32), _dev(out32), _dev(lam), r, S, N,
                                                     reference=_dev(R32), loss=loss, schedule=schedule))
    L_o, U_o = oracle.mse_loss_seed(out32, R32)
    G2_ref, gl2_ref = oracle.filter_backward(U_o, mean32, out32, lam, N, r, -30.0, S)
    assert np.isnan(_host(loss)[0]) and np.isnan(L_o)
    assert np.array_equal(np.isnan(G2), np.isnan(G2_ref)) and np.array_equal(np.isnan(gl2), np.isnan(gl2_ref))
    # the loss formed in the forward pass: the same NaN pattern
    out3, U3, loss3, gl3 = ops.filter_forward_loss(_dev(mean32), _dev(lam), r, _dev(R32), N, schedule=schedule)
    G3 = _host(ops.filter_backward_radiance(U3, _dev(lam), r, S, N, schedule=schedule))
    assert np.array_equal(np.isnan(_host(out3)), np.isnan(ref)) and np.isnan(_host(loss3)[0])
    assert np.array_equal(np.isnan(G3), np.isnan(G2_ref)) and np.array_equal(np.isnan(_host(gl3)), np.isnan(gl2_ref))


@pytest.mark.parametrize("schedule", [0] + SCHEDULES)
@pytest.mark.parametrize("W,H,N,r,S", [(130, 70, 4, 3, 8), (96, 54, 40, 5, 4), (333, 190, 3, 7, 16),
                                       (41, 9, 5, 15, 2), (67, 31, 1, 0, 2), (1, 1, 1, 2, 3), (96, 54, 4, 5, 64)])
def test_loss_in_forward_parity(W, H, N, r, S, schedule):
    # RAMLT_LOSS_IN_FORWARD: the forward pass forms out, U, the loss and dL/dlambda; the
    # adjoint then forms G from U alone. Against the oracle's chain, and against the plain
    # forward followed by the adjoint with the seed fused (the same results up to rounding).
    print(f"loss in forward W={W} H={H} N={N} r={r} S={S} schedule={schedule}", flush=True)
    _, mean32, lam = _filter_inputs(W, H, 4, N, seed=W * 5 + H)
    lam[:: max(1, N)] = -35.0
    ref32 = (mean32 * np.float32(0.9) + np.float32(0.05)).astype(np.float32)
    out, U, loss, gl = ops.filter_forward_loss(_dev(mean32), _dev(lam), r, _dev(ref32), N, schedule=schedule)
    G = ops.filter_backward_radiance(U, _dev(lam), r, S, N, schedule=schedule)
    out_o, _ = oracle.filter_forward(mean32, lam, N, r, -30.0)
    L_o, U_o = oracle.mse_loss_seed(out_o, ref32)
    G_o, gl_o = oracle.filter_backward(U_o, mean32, out_o, lam, N, r, -30.0, S)
    check("out", _host(out), out_o, filter_scale(mean32, lam, N, r, -30.0))
    n = out_o.size
    u_scale = 2.0 * (np.abs(out_o) + np.abs(ref32)) / n
    check("U", _host(U), U_o, u_scale)
    d = np.abs(out_o - ref32)
    check("loss", _host(loss)[0], L_o, L_o + (2 * d * (np.abs(out_o) + np.abs(ref32))).sum() / n)
    G_s, gl_s = backward_scales(u_scale, mean32, out_o, lam, N, r, -30.0, S)
    check("G", _host(G), G_o, G_s)
    check("grad_lambda", _host(gl), gl_o, gl_s)
    # the two-kernel split against the fused adjoint on the same GPU out
    loss2 = torch.zeros(1, dtype=torch.float64, device="cuda")
    G2, gl2 = ops.filter_backward(None, _dev(mean32), out, _dev(lam), r, S, N, reference=_dev(ref32), loss=loss2,
                                  schedule=schedule)
    check("G vs fused adjoint", _host(G), _host(G2), G_s)
    check("grad_lambda vs fused adjoint", _host(gl), _host(gl2), gl_s)
    assert abs(_host(loss)[0] - _host(loss2)[0]) <= 1e-12 * max(L_o, 1e-300)
