"""filter_backward_noalloc (the adjoint with the library's own device workspace, for callers
that cannot allocate) against filter_backward with a caller-allocated workspace, through the
C ABI: two calls in a row, the second on a smaller frame, then a batch; every output equal,
and both within the tolerance of the oracle."""

import numpy as np
import pytest
import torch

import oracle
from paper_2402_08273_amd import _abi, ops
from parity import backward_scales, check
from synth import make_frame, make_lambda, make_reference

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _frame_case(W, H, S, N, r, seed):
    rad, _ = make_frame(W, H, S, seed=seed, with_features=False)
    mean32 = oracle.stats_accumulate(rad, None, 0)["mean"].astype(np.float32)
    ref32 = make_reference(W, H, seed=seed + 1000, spp=16)
    lam = make_lambda(N, seed=seed)
    out32 = oracle.filter_forward(mean32, lam, N, r)[0].astype(np.float32)
    return mean32, ref32, lam, out32


def _descriptor(mean, out, ref, lam, N, r, S, G, gl, loss):
    f = ops.filter_frame(mean, lam, r, N)
    f.out, f.reference, f.loss = out.data_ptr(), ref.data_ptr(), loss.data_ptr()
    f.S = S
    f.grad_radiance, f.grad_lambda = G.data_ptr(), gl.data_ptr()
    return f


def _run_both(cases):
    """The same frames through filter_backward (torch workspace) and the no-alloc entry
    point; returns both sets of outputs."""
    results = []
    for use_static in (False, True):
        outs, frames = [], []
        for (mean32, ref32, lam, out32, N, r, S) in cases:
            t = dict(mean=_dev(mean32), ref=_dev(ref32), lam=_dev(lam), out=_dev(out32),
                     G=torch.full((3,) + mean32.shape[1:], np.nan, device="cuda"),
                     gl=torch.zeros(N * N, device="cuda"), loss=torch.zeros(1, dtype=torch.float64, device="cuda"))
            frames.append(_descriptor(t["mean"], t["out"], t["ref"], t["lam"], N, r, S, t["G"], t["gl"], t["loss"]))
            outs.append(t)
        table = (_abi.RamltFrame * len(frames))(*frames)
        dev_table = None
        keep = None
        if len(frames) > 1:
            import ctypes

            raw = bytes(ctypes.string_at(ctypes.addressof(table), ctypes.sizeof(table)))
            keep = torch.frombuffer(bytearray(raw), dtype=torch.uint8).cuda()
            dev_table = keep.data_ptr()
        stream = torch.cuda.current_stream().cuda_stream
        if use_static:
            _abi.filter_backward_noalloc(list(table), frames_dev=dev_table, stream=stream)
        else:
            need = _abi.workspace_size(list(table), _abi.OP_FILTER_BACKWARD)
            ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
            ptr = (ws.data_ptr() + 255) // 256 * 256
            _abi.filter_backward(list(table), frames_dev=dev_table, workspace=ptr, ws_bytes=need, stream=stream)
        torch.cuda.synchronize()
        results.append([{k: outs[i][k].cpu().numpy() for k in ("G", "gl", "loss")} for i in range(len(cases))])
        del keep
    return results


def _check_against_oracle(case, got):
    mean32, ref32, lam, out32, N, r, S = case
    L_o, U_o = oracle.mse_loss_seed(out32, ref32)
    G_o, gl_o = oracle.filter_backward(U_o, mean32, out32, lam, N, r, -30.0, S)
    u_scale = 2.0 * (np.abs(out32) + np.abs(ref32)) / out32.size
    G_s, gl_s = backward_scales(u_scale, mean32, out32, lam, N, r, -30.0, S)
    check("G", got["G"], G_o, G_s)
    check("grad_lambda", got["gl"], gl_o, gl_s)
    assert abs(got["loss"][0] - L_o) <= 1e-5 * L_o


def test_noalloc_adjoint_matches_the_workspace_form():
    # two calls in a row, the second on a smaller frame (the array keeps the first call's
    # partials: nothing of them may leak into the second), then a three-frame batch
    big = _frame_case(640, 360, 8, 20, 5, seed=3) + (20, 5, 8)
    small = _frame_case(130, 70, 4, 4, 3, seed=4) + (4, 3, 4)
    odd = _frame_case(41, 9, 2, 5, 2, seed=5) + (5, 2, 2)
    for name, cases in (("big", [big]), ("small", [small]), ("batch", [small, odd, big])):
        print("no-alloc case:", name, flush=True)
        ref_run, static_run = _run_both(cases)
        for i, case in enumerate(cases):
            a, b = ref_run[i], static_run[i]
            assert np.array_equal(a["G"], b["G"]), (name, i)
            # partial sums added in the same fixed order (atomics across the frames of a
            # batch that share nothing here): equal
            np.testing.assert_allclose(b["gl"], a["gl"], rtol=1e-6, atol=0)
            np.testing.assert_allclose(b["loss"], a["loss"], rtol=1e-12, atol=0)
            _check_against_oracle(case, b)


def test_noalloc_rejects_a_frame_beyond_its_workspace():
    f = ops.filter_frame(torch.zeros((3, 4, 4), device="cuda"), torch.zeros(4, device="cuda"), 3, 2)
    f.W, f.H, f.n_regions = 32768, 32768, 1  # 4 M tiles of partial sums: beyond 4 MiB
    f.out = f.reference = f.grad_radiance = f.mean
    f.S = 1
    assert _abi.workspace_size([f], _abi.OP_FILTER_BACKWARD) > 4 << 20
    lib = _abi.load()
    st = lib.filter_backward_noalloc((_abi.RamltFrame * 1)(f), None, 1, None)
    assert st == _abi.RAMLT_EWORKSPACE and "workspace" in _abi.last_error()
