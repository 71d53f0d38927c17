"""Batched execution: many frames of uneven size and sample count processed by one launch
per operation (per radius for the filter), with the whole forward + backward step
capturable in a HIP graph.

``FrameBatch`` owns the output buffers, the host descriptor table, its device copy and
the workspace in which each batched launch plans its tiles on the device. Every
operation is one call into ``libramlt.so``; torch only provides memory, streams and
graph capture.
"""

import ctypes
from typing import List, Optional, Sequence

import torch

from . import _abi
from ._abi import RamltFrame
from .ops import LAMBDA_MIN_DEFAULT


class FrameInput:
    """Inputs of one frame: radiance [3,S,H,W] (fp32), optional features [7,S,H,W]
    (fp32/fp16), optional reference [3,H,W] (for the MSE seed), the lambda table
    (shared tensors are allowed) and the filter radius."""

    def __init__(self, radiance, features=None, reference=None, lam=None, radius=5, n_regions=20,
                 lambda_min=LAMBDA_MIN_DEFAULT, max_lag=8, grad_lambda=None, schedule=0):
        self.radiance = radiance
        self.features = features
        self.reference = reference
        self.lam = lam
        self.radius = int(radius)
        self.n_regions = int(n_regions)
        self.lambda_min = float(lambda_min)
        self.max_lag = int(max_lag)
        self.grad_lambda = grad_lambda
        self.schedule = int(schedule)  # ramlt_frame.flags: filter tile shape / direct gather


class FrameBatch:
    """Outputs per frame: mean/var/tau [3,H,W], feat_mean/feat_var [7,H,W], out [3,H,W],
    grad_radiance [3,H,W] (dL/dg for every sample); grad_lambda (per frame, or shared
    when the frames share one tensor), and one fp64 loss = sum over frames of each
    frame's MSE."""

    def __init__(self, frames: Sequence[FrameInput], device="cuda", loss_in_forward=False):
        """``loss_in_forward``: the forward launch also forms the MSE seed (U, kept per
        frame as ``grad_out``), the loss and dL/dlambda (RAMLT_LOSS_IN_FORWARD); the
        backward launch then forms the radiance gradient only. Every frame needs a
        reference."""
        if not frames:
            raise ValueError("empty batch")
        self.device = torch.device(device)
        self.inputs = list(frames)
        self.loss_in_forward = bool(loss_in_forward)
        if self.loss_in_forward and any(fi.reference is None for fi in self.inputs):
            raise ValueError("loss_in_forward needs a reference for every frame")
        f32 = dict(device=self.device, dtype=torch.float32)
        self.loss = torch.zeros(1, device=self.device, dtype=torch.float64)
        self.outputs = []
        descs: List[RamltFrame] = []
        # frames without a given gradient buffer get views of one flat tensor, so that
        # zeroing all of them is one fill kernel
        own = [fi.lam.numel() for fi in self.inputs if fi.grad_lambda is None]
        self._grad_flat = torch.zeros(max(sum(own), 1), **f32)
        grads = [self._grad_flat]
        off = 0
        for fi in self.inputs:
            rad = fi.radiance
            _, S, H, W = rad.shape
            o = {
                "mean": torch.empty((3, H, W), **f32),
                "var": torch.empty((3, H, W), **f32),
                "tau": torch.empty((3, H, W), **f32),
                "out": torch.empty((3, H, W), **f32),
                "grad_radiance": torch.empty((3, H, W), **f32),
            }
            if fi.features is not None:
                o["feat_mean"] = torch.empty((7, H, W), **f32)
                o["feat_var"] = torch.empty((7, H, W), **f32)
            if fi.grad_lambda is not None:
                gl = fi.grad_lambda
                if all(gl is not g for g in grads):
                    grads.append(gl)
            else:
                gl = self._grad_flat[off:off + fi.lam.numel()]
                off += fi.lam.numel()
            o["grad_lambda"] = gl
            d = RamltFrame()
            d.W, d.H, d.S, d.max_lag = W, H, S, fi.max_lag
            d.radiance = rad.data_ptr()
            d.rad_stride_c, d.rad_stride_s, d.rad_stride_y = rad.stride(0), rad.stride(1), rad.stride(2)
            if fi.features is not None:
                ft = fi.features
                d.features = ft.data_ptr()
                d.feat_stride_c, d.feat_stride_s, d.feat_stride_y = ft.stride(0), ft.stride(1), ft.stride(2)
                d.feat_dtype = _abi.RAMLT_F16 if ft.dtype == torch.float16 else _abi.RAMLT_F32
                d.feat_mean, d.feat_var = o["feat_mean"].data_ptr(), o["feat_var"].data_ptr()
            d.mean, d.var, d.tau = o["mean"].data_ptr(), o["var"].data_ptr(), o["tau"].data_ptr()
            d.lambda_ = fi.lam.data_ptr()
            d.n_regions, d.radius, d.lambda_min = fi.n_regions, fi.radius, fi.lambda_min
            d.flags = fi.schedule | (_abi.RAMLT_LOSS_IN_FORWARD if self.loss_in_forward else 0)
            d.out = o["out"].data_ptr()
            if self.loss_in_forward:
                o["grad_out"] = torch.empty((3, H, W), **f32)
                d.grad_out = o["grad_out"].data_ptr()
            if fi.reference is not None:
                d.reference = fi.reference.data_ptr()
                d.loss = self.loss.data_ptr()
            d.grad_radiance = o["grad_radiance"].data_ptr()
            d.grad_lambda = gl.data_ptr()
            self.outputs.append(o)
            descs.append(d)
        self._grads = grads
        self.n = len(descs)
        self.table = (RamltFrame * self.n)(*descs)
        self._graph: Optional[torch.cuda.CUDAGraph] = None
        self._upload()

    def _upload(self):
        """Device copy of the descriptor table and a workspace for every operation."""
        raw = bytes(ctypes.string_at(ctypes.addressof(self.table), ctypes.sizeof(self.table)))
        self.table_dev = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(self.device)
        ws = max(_abi.workspace_size(list(self.table), op) for op in
                 (_abi.OP_STATS, _abi.OP_FILTER_FORWARD, _abi.OP_LOSS_SEED, _abi.OP_FILTER_BACKWARD))
        self.workspace = torch.empty(max(ws, 256) + 256, device=self.device, dtype=torch.uint8)
        base = self.workspace.data_ptr()
        self.ws_ptr = (base + 255) // 256 * 256
        self.ws_bytes = max(ws, 256)

    def tune(self, **kw):
        """Choose the filter's launch schedule (tile shape, window schedule) and the
        statistics pass's launch size for this batch by timing the candidates on its own
        frames (:mod:`.tune`, cached by shape), write them into every descriptor and rebuild
        the device table and workspace. Needs the statistics of the frames (run ``stats()``
        first); clears the gradient and loss accumulators. Call before ``capture()``.
        Returns the filter schedule; the statistics launch size is ``self.stats_launch``."""
        from . import tune as _tune

        if self._graph is not None:
            raise RuntimeError("tune() before capture()")
        best = _tune.tune_table(self.table, device=self.device, zero=self._grads + [self.loss], **kw)
        self._upload()
        self.stats_launch = _tune.tune_stats(self.table, device=self.device,
                                             table_dev=self.table_dev if self.n > 1 else None,
                                             cache=kw.get("cache"), force=kw.get("force", False))
        self._upload()
        return best

    # ------------------------------------------------------------------ single ops
    def _call(self, name):
        lib = _abi.load()
        st = getattr(lib, name)(self.table, self.table_dev.data_ptr() if self.n > 1 else None, self.n,
                                self.ws_ptr, self.ws_bytes, torch.cuda.current_stream(self.device).cuda_stream)
        if st != _abi.RAMLT_OK:
            raise _abi.RamltError(st, _abi.last_error())

    def stats(self):
        self._call("stats_accumulate")

    def forward(self):
        self._call("filter_forward")

    def zero_grads(self):
        for g in self._grads:
            g.zero_()
        self.loss.zero_()

    def backward(self):
        """Fused MSE seed + adjoint (every frame needs a reference); with loss_in_forward,
        the radiance gradient from the seed the forward launch formed."""
        self._call("filter_backward")

    def step(self):
        """stats -> filter -> (zero accumulators) -> fused loss seed + adjoint; with
        loss_in_forward: stats -> (zero accumulators) -> filter with the seed, the loss and
        dL/dlambda -> radiance gradient."""
        self.stats()
        if self.loss_in_forward:
            self.zero_grads()
            self.forward()
        else:
            self.forward()
            self.zero_grads()
        self.backward()

    # ------------------------------------------------------------------ graphs
    def capture(self, warmup=1):
        """Capture one step() into a HIP graph (all descriptors and the workspace are
        already device-resident, so the graph contains only kernel launches)."""
        s = torch.cuda.Stream(device=self.device)
        s.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(s):
            for _ in range(warmup):
                self.step()
        torch.cuda.current_stream(self.device).wait_stream(s)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.step()
        self._graph = g
        return g

    def replay(self):
        if self._graph is None:
            raise RuntimeError("capture() first")
        self._graph.replay()
