"""GPU tests of the fused loss seed + adjoint, the batched launches (against
single-frame launches and the oracle), HIP graph replay (against eager), and the
autograd binding."""

import numpy as np
import pytest
import torch

import oracle
from paper_2402_08273_amd import _abi, ops
from paper_2402_08273_amd.batch import FrameBatch, FrameInput
from parity import backward_scales, check, filter_scale, stats_scales
from synth import make_frame, make_lambda, make_reference

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _h(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _oracle_chain(rad, feats, ref, lam, N, r, S):
    o = oracle.stats_accumulate(rad, feats, 8)
    out_o, _ = oracle.filter_forward(o["mean"], lam, N, r)
    L_o, U_o = oracle.mse_loss_seed(out_o, ref)
    G_o, gl_o = oracle.filter_backward(U_o, o["mean"], out_o, lam, N, r, -30.0, S)
    return o, out_o, L_o, U_o, G_o, gl_o


def _check_chain(name, rad, feats, ref, lam, N, r, S, st, out, loss, G, gl):
    o, out_o, L_o, U_o, G_o, gl_o = _oracle_chain(rad, feats, ref, lam, N, r, S)
    sc = stats_scales(rad, o)
    check(name + " mean", st["mean"], o["mean"], sc["mean"])
    check(name + " var", st["var"], o["var"], sc["var"])
    check(name + " tau", st["tau"], o["tau"], sc["tau"])
    check(name + " out", out, out_o, filter_scale(o["mean"], lam, N, r, -30.0))
    n = out_o.size
    u_scale = 2.0 * (np.abs(out_o) + np.abs(ref)) / n
    if loss is not None:
        d = np.abs(out_o - ref)
        check(name + " loss", loss, L_o, L_o + (2 * d * (np.abs(out_o) + np.abs(ref))).sum() / n)
    G_s, gl_s = backward_scales(u_scale, o["mean"], out_o, lam, N, r, -30.0, S)
    check(name + " G", G, G_o, G_s)
    if gl is not None:
        check(name + " grad_lambda", gl, gl_o, gl_s)
    return gl_s


@pytest.mark.parametrize("W,H,S,N,r", [(128, 128, 16, 20, 3), (97, 61, 8, 4, 5), (45, 30, 5, 20, 2)])
def test_fused_loss_seed_and_adjoint(W, H, S, N, r):
    rad, feats = make_frame(W, H, S, seed=W + S)
    ref = make_reference(W, H, seed=1000 + W, spp=32)
    lam = make_lambda(N, seed=99)
    st = ops.stats(_dev(rad), _dev(feats), 8)
    out = ops.filter_forward(st.mean, _dev(lam), r, N)
    loss = torch.zeros(1, device="cuda", dtype=torch.float64)
    G, gl = ops.filter_backward(None, st.mean, out, _dev(lam), r, S, N, reference=_dev(ref), loss=loss)
    _check_chain("fused", rad, feats, ref, lam, N, r, S,
                 {"mean": _h(st.mean), "var": _h(st.var), "tau": _h(st.tau)}, _h(out), _h(loss)[0], _h(G), _h(gl))


def _batch_inputs(specs, shared_lam):
    shared_grad = torch.zeros_like(shared_lam)
    frames, host = [], []
    for i, (W, H, S, r, fdt) in enumerate(specs):
        rad, feats = make_frame(W, H, S, seed=10 + i, frame=i,
                                feature_dtype=fdt if fdt is not None else np.float32,
                                with_features=fdt is not None)
        ref = make_reference(W, H, seed=2000 + i, frame=i, spp=16)
        host.append((rad, feats, ref, r))
        frames.append(FrameInput(_dev(rad), None if feats is None else _dev(feats), _dev(ref), shared_lam,
                                 radius=r, n_regions=20, grad_lambda=shared_grad))
    return frames, host


SPECS = [(37, 23, 3, 3, np.float32), (64, 40, 16, 3, None), (128, 128, 4, 5, np.float16),
         (50, 70, 33, 5, np.float32), (200, 90, 1, 3, None), (96, 54, 64, 3, np.float16)]


def test_batched_matches_single_frames_and_oracle():
    lam = make_lambda(20, seed=99)
    lam_d = _dev(lam)
    frames, host = _batch_inputs(SPECS, lam_d)
    b = FrameBatch(frames)
    b.step()
    torch.cuda.synchronize()
    # single-frame launches of the same ops, frame by frame
    loss_total = 0.0
    gl_sum = np.zeros(400)
    gl_scale = np.zeros(400)
    for i, (rad, feats, ref, r) in enumerate(host):
        o = b.outputs[i]
        S = rad.shape[1]
        st = ops.stats(frames[i].radiance, frames[i].features, 8)
        out = ops.filter_forward(st.mean, lam_d, r, 20)
        assert np.array_equal(_h(st.mean), _h(o["mean"]))
        assert np.array_equal(_h(st.tau), _h(o["tau"]))
        assert np.array_equal(_h(out), _h(o["out"]))
        if feats is not None:
            assert np.array_equal(_h(st.feat_var), _h(o["feat_var"]))
        gl_s = _check_chain(f"frame {i}", rad, feats, ref, lam, 20, r, S,
                            {k: _h(o[k]) for k in ("mean", "var", "tau")}, _h(o["out"]), None,
                            _h(o["grad_radiance"]), None)
        ch = _oracle_chain(rad, feats, ref, lam, 20, r, S)
        loss_total += ch[2]
        gl_sum += ch[5]
        gl_scale += gl_s
    # shared lambda: gradients and losses of all frames accumulate
    check("batch grad_lambda", _h(o["grad_lambda"]), gl_sum, gl_scale)
    assert abs(_h(b.loss)[0] - loss_total) <= 1e-5 * loss_total


def test_batched_stats_launch_sizes_give_the_same_results():
    # the batch's work units run in launches of v workgroups per compute unit, or in one
    # launch; the statistics are the same bits either way
    lam_d = _dev(make_lambda(20, seed=99))
    frames, _ = _batch_inputs(SPECS, lam_d)
    b = FrameBatch(frames)
    got = {}
    for v in (1, 3, _abi.RAMLT_STATS_ONE_LAUNCH):
        for d in b.table:
            d.flags = (d.flags & ~_abi.RAMLT_STATS_WG_MASK) | (v << _abi.RAMLT_STATS_WG_SHIFT)
        b._upload()
        b.stats()
        got[v] = [{k: _h(o[k]) for k in ("mean", "var", "tau", "feat_mean", "feat_var") if o.get(k) is not None}
                  for o in b.outputs]
    for v, frames_v in got.items():
        for i, (a, ref) in enumerate(zip(frames_v, got[1])):
            for k in ref:
                assert np.array_equal(a[k], ref[k], equal_nan=True), (v, i, k)


def test_batched_loss_in_forward_matches_oracle():
    # the six uneven frames (fp32 / fp16 / no features, S from 1 to 64, shared lambda and
    # gradient) with the loss formed in the forward launch
    lam = make_lambda(20, seed=99)
    lam_d = _dev(lam)
    frames, host = _batch_inputs(SPECS, lam_d)
    b = FrameBatch(frames, loss_in_forward=True)
    b.step()
    torch.cuda.synchronize()
    loss_total, gl_sum, gl_scale = 0.0, np.zeros(400), np.zeros(400)
    for i, (rad, feats, ref, r) in enumerate(host):
        o = b.outputs[i]
        S = rad.shape[1]
        gl_s = _check_chain(f"frame {i}", rad, feats, ref, lam, 20, r, S,
                            {k: _h(o[k]) for k in ("mean", "var", "tau")}, _h(o["out"]), None,
                            _h(o["grad_radiance"]), None)
        ch = _oracle_chain(rad, feats, ref, lam, 20, r, S)
        n = ch[1].size
        check(f"frame {i} U", _h(o["grad_out"]), ch[3], 2.0 * (np.abs(ch[1]) + np.abs(ref)) / n)
        loss_total += ch[2]
        gl_sum += ch[5]
        gl_scale += gl_s
    check("batch grad_lambda", _h(b.outputs[0]["grad_lambda"]), gl_sum, gl_scale)
    assert abs(_h(b.loss)[0] - loss_total) <= 1e-5 * loss_total


# Frames large enough for region-aligned tiling (>= 16 N x 4 N pixels), each with its own
# lambda table, grid size and gradient buffer; three radii, so the batch runs three plans.
ALIGNED_SPECS = [(96, 40, 4, 3, 4), (130, 37, 8, 5, 4), (64, 16, 2, 0, 4), (200, 90, 5, 5, 6),
                 (320, 80, 3, 3, 20)]


@pytest.mark.parametrize("loss_in_forward", [False, True])
def test_batched_region_aligned_frames(loss_in_forward):
    frames, host = [], []
    for i, (W, H, S, r, N) in enumerate(ALIGNED_SPECS):
        rad, _ = make_frame(W, H, S, seed=30 + i, frame=i, with_features=False)
        ref = make_reference(W, H, seed=3000 + i, frame=i, spp=16)
        lam = make_lambda(N, seed=50 + i)
        host.append((rad, ref, lam, N, r))
        # mixed launch schedules: tile kinds and the direct gather inside one batch
        sched = [0, _abi.RAMLT_TILE_32X16, _abi.RAMLT_TILE_64X8, _abi.RAMLT_SCHED_DIRECT,
                 _abi.RAMLT_TILE_32X16 | _abi.RAMLT_SCHED_DIRECT][i]
        frames.append(FrameInput(_dev(rad), None, _dev(ref), _dev(lam), radius=r, n_regions=N, schedule=sched))
    b = FrameBatch(frames, loss_in_forward=loss_in_forward)
    b.step()
    torch.cuda.synchronize()
    loss_total = 0.0
    for i, (rad, ref, lam, N, r) in enumerate(host):
        o = b.outputs[i]
        S = rad.shape[1]
        _check_chain(f"aligned frame {i}", rad, None, ref, lam, N, r, S,
                     {k: _h(o[k]) for k in ("mean", "var", "tau")}, _h(o["out"]), None,
                     _h(o["grad_radiance"]), _h(o["grad_lambda"]))
        loss_total += _oracle_chain(rad, None, ref, lam, N, r, S)[2]
    assert abs(_h(b.loss)[0] - loss_total) <= 1e-5 * loss_total


def test_single_frame_adjoint_is_deterministic():
    # region-aligned frame: dL/dlambda and the loss are per-tile partials added in a fixed order
    W, H, S, N, r = 400, 120, 4, 20, 4
    rad, _ = make_frame(W, H, S, seed=7, with_features=False)
    ref = _dev(make_reference(W, H, seed=1007, spp=16))
    lam = _dev(make_lambda(N, seed=99))
    st = ops.stats(_dev(rad), None, 8)
    out = ops.filter_forward(st.mean, lam, r, N)
    runs = []
    for _ in range(3):
        loss = torch.zeros(1, device="cuda", dtype=torch.float64)
        G, gl = ops.filter_backward(None, st.mean, out, lam, r, S, N, reference=ref, loss=loss)
        runs.append((_h(G).copy(), _h(gl).copy(), _h(loss).copy()))
    for G, gl, loss in runs[1:]:
        assert np.array_equal(G, runs[0][0])
        assert np.array_equal(gl, runs[0][1])
        assert np.array_equal(loss, runs[0][2])


@pytest.mark.parametrize("loss_in_forward", [False, True])
def test_graph_replay_matches_eager(loss_in_forward):
    lam_d = _dev(make_lambda(20, seed=99))
    frames, _ = _batch_inputs(SPECS[:4], lam_d)
    b = FrameBatch(frames, loss_in_forward=loss_in_forward)
    b.step()
    torch.cuda.synchronize()
    eager = [{k: _h(v).copy() for k, v in o.items()} for o in b.outputs]
    eager_loss = _h(b.loss)[0]
    b.capture()
    for rep in range(3):
        # eager work and a synchronisation between replays
        torch.cuda.synchronize()
        junk = torch.randn(1000, device="cuda").sum()
        b.replay()
        torch.cuda.synchronize()
        for i, o in enumerate(b.outputs):
            for k in ("mean", "var", "tau", "out") + (("grad_out",) if loss_in_forward else ()):
                assert np.array_equal(_h(o[k]), eager[i][k]), (rep, i, k)
            np.testing.assert_allclose(_h(o["grad_radiance"]), eager[i]["grad_radiance"], rtol=0, atol=0)
            np.testing.assert_allclose(_h(o["grad_lambda"]), eager[i]["grad_lambda"], rtol=1e-5, atol=1e-12)
        assert abs(_h(b.loss)[0] - eager_loss) <= 1e-12 * abs(eager_loss)
        del junk


def test_autograd_regional_filter():
    W, H, S, N, r = 70, 45, 8, 5, 3
    rad, feats = make_frame(W, H, S, seed=3)
    ref = make_reference(W, H, seed=1003, spp=16)
    lam = make_lambda(N, seed=99)
    rad_t = _dev(rad).requires_grad_(True)
    lam_t = _dev(lam).requires_grad_(True)
    out = ops.RegionalFilter.apply(rad_t, _dev(feats), lam_t, r, N)
    loss = ops.MSELoss.apply(out, _dev(ref))
    loss.backward()
    _, out_o, L_o, _, G_o, gl_o = _oracle_chain(rad, feats, ref, lam, N, r, S)
    assert abs(float(loss.detach()) - L_o) <= 1e-5 * L_o
    g = _h(rad_t.grad)
    assert g.shape == rad.shape
    # every sample of a pixel gets the same gradient
    assert np.array_equal(g[:, 0], g[:, S - 1])
    o = oracle.stats_accumulate(rad, None, 0)
    u_scale = 2.0 * (np.abs(out_o) + np.abs(ref)) / out_o.size
    G_s, gl_s = backward_scales(u_scale, o["mean"], out_o, lam, N, r, -30.0, S)
    check("autograd G", g[:, 0], G_o, G_s)
    check("autograd grad_lambda", _h(lam_t.grad), gl_o, gl_s)


def test_tuned_batch_matches_oracle(tmp_path):
    # the autotuner picks a schedule by timing, writes it into the batch, and the tuned
    # step still matches the oracle; a second batch of the same shapes reads the cache
    from paper_2402_08273_amd import tune

    cache = tune.TuneCache(str(tmp_path / "tune.json"))
    lam = make_lambda(20, seed=99)
    lam_d = _dev(lam)
    frames, host = _batch_inputs(SPECS[:3], lam_d)
    b = FrameBatch(frames)
    b.stats()
    best = b.tune(cache=cache, reps=3, warmup=1)
    assert best in tune.CANDIDATES
    assert all(d.flags & tune.SCHEDULE_BITS == best for d in b.table)
    key = tune.workload_key(b.table, tune.device_arch())
    assert cache.record(key)["schedule"] == best and len(cache.record(key)["ms"]) == len(tune.CANDIDATES)
    # the statistics launch size, timed on the same frames, is in bits 4-7 of every descriptor
    assert b.stats_launch in tune.STATS_CANDIDATES
    assert all((d.flags & _abi.RAMLT_STATS_WG_MASK) >> _abi.RAMLT_STATS_WG_SHIFT == b.stats_launch for d in b.table)
    skey = tune.stats_workload_key(b.table, tune.device_arch())
    assert cache.record(skey)["schedule"] == b.stats_launch
    assert len(cache.record(skey)["ms"]) == len(tune.STATS_CANDIDATES)
    b.step()
    torch.cuda.synchronize()
    gl_sum, gl_scale, loss_total = np.zeros(400), np.zeros(400), 0.0
    for i, (rad, feats, ref, r) in enumerate(host):
        o = b.outputs[i]
        gl_s = _check_chain(f"tuned frame {i}", rad, feats, ref, lam, 20, r, rad.shape[1],
                            {k: _h(o[k]) for k in ("mean", "var", "tau")}, _h(o["out"]), None,
                            _h(o["grad_radiance"]), None)
        ch = _oracle_chain(rad, feats, ref, lam, 20, r, rad.shape[1])
        loss_total += ch[2]
        gl_sum += ch[5]
        gl_scale += gl_s
    check("tuned batch grad_lambda", _h(b.outputs[0]["grad_lambda"]), gl_sum, gl_scale)
    assert abs(_h(b.loss)[0] - loss_total) <= 1e-5 * loss_total
    frames2, _ = _batch_inputs(SPECS[:3], lam_d)
    b2 = FrameBatch(frames2)
    b2.stats()
    assert b2.tune(cache=cache) == best  # from the cache, no timing
