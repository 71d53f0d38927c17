"""Throughput of the per-pixel chain statistics + regional reconstruction filter path on one
MI355X, at 1920x1080 with 64 spp (fp32 RGB radiance + albedo/normal/depth features), 11x11
window (radius 5), 20x20 region grid.

One step = the whole hot path over one frame already resident in HBM:
  stats_accumulate -> filter_forward forming out, the MSE loss seed U (vs a 4096-spp
  reference), the loss and dL/dlambda -> filter_backward forming the gradient of every
  radiance sample from U.
`value` is filtered Mpixel/s of that fwd+bwd step. Reported beside it: the forward-only
rate (stats + filter), the step with the seed fused into the adjoint or in a separate
loss_seed kernel, the 32-frame batch of uneven frames replayed as one HIP graph per step,
the 3840x2160 / 256 spp / fp16 feature frame with a 15x15 window, and the rows beyond the
filter. Inputs are synthetic and seeded (synth/), generated on the GPU before timing.
Timed regions are K back-to-back steps between two synchronisations (defaults K = 200,
W = 20): a timed region carries a fixed start-up cost of about 1 ms on MI355X, which K
spreads over the steps.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-extra]
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# the timed steps whose launches are bracketed by HIP events (every MARK_EVERY-th)
MARK_EVERY = 8


def parse():
    from synth.workloads import HD, N_REGIONS

    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--width", type=int, default=HD.W)
    p.add_argument("--height", type=int, default=HD.H)
    p.add_argument("--spp", type=int, default=HD.S)
    p.add_argument("--radius", type=int, default=HD.radius)
    p.add_argument("--regions", type=int, default=N_REGIONS)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-extra", action="store_true", help="skip the batched and 4K measurements")
    p.add_argument("--no-tune", action="store_true",
                   help="use the library's default filter schedule instead of the autotuned one")
    p.add_argument("--only", choices=["batched", "uhd", "adapt", "quadtree", "perturb", "rrmse", "lens", "small",
                                      "leaf_grad", "copy"], default=None,
                   help="measure only the 32-frame batch or only the 4K frame and print that object "
                        "(for profiling one workload)")
    p.add_argument("--cpu-rows", type=int, default=0, help="rows of the frame the oracle times (0 = auto)")
    p.add_argument("--traffic", type=str, default=os.path.join(ROOT, "profiles", "hbm_traffic.json"),
                   help="rocprofv3 HBM byte counts of the measured kernels (JSON records); a record is "
                        "ignored if a source it names changed since it was taken")
    p.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                   help="only run a plain device-to-device copy of MIB MiB (counter calibration) and exit")
    return p.parse_args()


def calibrate_copy(mib):
    """A plain copy kernel of known size, for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE."""
    import torch

    n = mib * (1 << 20) // 4
    src = torch.ones(n, device="cuda:0", dtype=torch.float32)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": 3}), flush=True)


TRAFFIC_RECORDS = os.path.join(ROOT, "profiles", "hbm_traffic.json")


def measured_traffic(path, key, field="bytes_per_launch"):
    """HBM bytes per launch of the kernel of workload ``key`` from the committed rocprofv3
    counts (FETCH_SIZE + WRITE_SIZE, scaled by the copy calibration), or None if there is no
    record for it or a source it names has changed since the counters were taken. ``field``
    picks another counted value of the record (e.g. VALU wave instructions per launch)."""
    import hashlib

    if not path or not os.path.exists(path):
        return None
    for rec in json.load(open(path))["records"]:
        if rec["key"] != key or field not in rec:
            continue
        h = hashlib.sha256()
        for src in rec["sources"]:
            h.update(open(os.path.join(ROOT, src), "rb").read())
        return rec[field] if h.hexdigest()[:16] == rec["sources_sha256_16"] else None
    return None


# VALU issue ceiling of MI355X: 256 CUs x 4 SIMDs, one wave64 VALU instruction per SIMD per
# 4 cycles at 2.4 GHz
VALU_PEAK_GINST_S = 256 * 4 * 2.4 / 4


def valu_roofline(insts, ms, note):
    """Roofline object against the VALU issue ceiling, reported beside a kernel's HBM one:
    its counted VALU wave instructions per launch (rocprofv3 SQ_INSTS_VALU, committed record)
    over the measured time. A high fraction says issue could bind; whether it does shows
    when fewer instructions shorten the kernel (for the lens step and the direction
    perturbation they did not: their counted bytes already move at a device copy's rate)."""
    if insts is None:
        return None
    g = insts / (ms * 1e-3) / 1e9
    return {"bound": "alu", "achieved": round(g, 1), "peak": VALU_PEAK_GINST_S, "unit": "G VALU wave-instructions/s",
            "frac": round(g / VALU_PEAK_GINST_S, 4), "valu_insts": int(insts), "covers": note}


def stats_bytes(P, S, feat_bytes=4):
    # every sample read once (3 radiance fp32 + 7 features) + 23 fp32 output planes
    return P * S * (3 * 4 + 7 * feat_bytes) + P * 23 * 4


# the filter's part of a step, 72 B per pixel in both forms: forward with the loss (mean,
# reference read; out, U written) + radiance adjoint (U read, G written), or plain forward
# (mean read, out written) + adjoint with the seed fused (mean, out, reference read; G written)
FILTER_STEP_BYTES_PER_PX = 24 + 48


class SingleChain:
    """Descriptors and buffers of one frame's step, built once; ``step()`` only launches:
    stats -> filter -> zero the accumulators -> fused loss seed + adjoint (or, unfused,
    loss_seed writing U and the adjoint reading it)."""

    def __init__(self, W, H, S, r, N, seed, frame=0, fp16_features=False, tune=True):
        import torch

        from paper_2402_08273_amd import _abi, ops
        from synth import gpu as sgpu
        from synth import make_lambda
        from synth.workloads import LAMBDA_SEED, MAX_LAG, REFERENCE_SPP

        dev = torch.device("cuda:0")
        self.W, self.H, self.S, self.r, self.N = W, H, S, r, N
        self.P = W * H
        self.feat_bytes = 2 if fp16_features else 4
        # inputs (untimed): seeded synthetic frame, reference, lambda table
        self.rad, self.feat = sgpu.make_frame(W, H, S, seed=seed, frame=frame,
                                              feature_dtype=torch.float16 if fp16_features else torch.float32)
        self.ref = sgpu.make_reference(W, H, seed=seed + 1000, frame=frame, spp=REFERENCE_SPP)
        self.lam = torch.from_numpy(make_lambda(N, seed=LAMBDA_SEED)).to(dev)
        f32 = dict(device=dev, dtype=torch.float32)
        mean, var, tau = (torch.empty((3, H, W), **f32) for _ in range(3))
        fmean, fvar = torch.empty((7, H, W), **f32), torch.empty((7, H, W), **f32)
        self.out, self.U, self.G = (torch.empty((3, H, W), **f32) for _ in range(3))
        # the adjoint's two accumulators share one buffer, so a step clears them with one fill
        acc_bytes = (N * N * 4 + 7) // 8 * 8
        self.acc = torch.zeros(acc_bytes + 8, device=dev, dtype=torch.uint8)
        self.grad_lam = self.acc[:N * N * 4].view(torch.float32)
        self.loss = self.acc[acc_bytes:].view(torch.float64)
        st_out = ops.Stats(mean, var, tau, None, fmean, fvar)
        fs, _ = ops.stats_frame(self.rad, self.feat, MAX_LAG, st_out, with_lag_corr=False)
        ff = ops.filter_frame(mean, self.lam, r, N)
        ff.out, ff.S = self.out.data_ptr(), S
        ff.reference, ff.loss = self.ref.data_ptr(), self.loss.data_ptr()
        ff.grad_radiance, ff.grad_lambda = self.G.data_ptr(), self.grad_lam.data_ptr()
        # fused: the MSE seed is formed inside the adjoint (grad_out NULL)
        fu = _abi.RamltFrame.from_buffer_copy(ff)
        fu.grad_out = self.U.data_ptr()  # unfused variant: loss_seed writes U, the adjoint reads it
        # loss in the forward pass: the forward writes out and U and accumulates the loss and
        # dL/dlambda; the adjoint forms G from U
        fl = _abi.RamltFrame.from_buffer_copy(fu)
        fl.flags = _abi.RAMLT_LOSS_IN_FORWARD
        self.stream = torch.cuda.current_stream()
        self.sh = self.stream.cuda_stream
        self.tabs = (_abi.RamltFrame * 1)(fs)
        self.tabf = (_abi.RamltFrame * 1)(ff)
        self.tabu = (_abi.RamltFrame * 1)(fu)
        self.tabl = (_abi.RamltFrame * 1)(fl)
        self.lib = _abi.load()
        self._abi = _abi
        if tune:
            # filter schedule (tile shape, window schedule) timed on this frame for each form of
            # the step, untimed here
            from paper_2402_08273_amd import tune as _tune

            # statistics launch size, then the filter schedule on the frame's statistics
            _tune.tune_stats(self.tabs)
            self.call0(self.lib.stats_accumulate, self.tabs)
            _tune.tune_table(self.tabf, zero=[self.acc])
            self.tabu[0].flags = self.tabf[0].flags
            _tune.tune_table(self.tabl, zero=[self.acc])
        # the filter's workspace (per-tile partial sums), allocated once
        need = max(_abi.workspace_size([t[0]], op) for t in (self.tabf, self.tabl)
                   for op in (_abi.OP_FILTER_FORWARD, _abi.OP_FILTER_BACKWARD))
        self.ws_t = torch.empty(need + 256, device=dev, dtype=torch.uint8)
        self.ws_ptr, self.ws_bytes = (self.ws_t.data_ptr() + 255) // 256 * 256, need
        torch.cuda.synchronize()

    def call0(self, fn, tab):
        st = fn(tab, None, 1, None, 0, self.sh)
        if st != 0:
            raise RuntimeError(self._abi.last_error())

    def call(self, fn, tab):
        st = fn(tab, None, 1, self.ws_ptr, self.ws_bytes, self.sh)
        if st != 0:
            raise RuntimeError(self._abi.last_error())

    def stats(self):
        self.call(self.lib.stats_accumulate, self.tabs)

    def forward(self):
        self.call(self.lib.filter_forward, self.tabf)

    def step(self, marks=None, form="loss_in_forward"):
        """One step: stats -> filter -> loss seed -> adjoint. ``form``: "loss_in_forward" (the
        forward forms out, U, the loss and dL/dlambda; the adjoint G), "fused" (plain forward;
        the seed fused into the adjoint) or "unfused" (plain forward, loss_seed, adjoint)."""
        if marks is not None:
            marks[0].record(self.stream)
        self.stats()
        if marks is not None:
            marks[1].record(self.stream)
        if form == "loss_in_forward":
            self.acc.zero_()
            self.call(self.lib.filter_forward, self.tabl)
            if marks is not None:
                marks[2].record(self.stream)
            self.call(self.lib.filter_backward, self.tabl)
            if marks is not None and len(marks) > 3:
                marks[3].record(self.stream)
            return
        self.forward()
        if marks is not None:
            marks[2].record(self.stream)
        self.acc.zero_()
        if form == "fused":
            self.call(self.lib.filter_backward, self.tabf)
        else:
            self.call(self.lib.loss_seed, self.tabu)
            self.call(self.lib.filter_backward, self.tabu)

    def one_call_table(self):
        """The step's descriptor for stats_filter_step: the statistics fields and launch size of
        the stats descriptor, the filter fields and schedule of the loss-in-forward one."""
        from paper_2402_08273_amd import _abi

        f = _abi.RamltFrame.from_buffer_copy(self.tabl[0])
        s = self.tabs[0]
        for name in ("S", "max_lag", "radiance", "rad_stride_c", "rad_stride_s", "rad_stride_y", "features",
                     "feat_stride_c", "feat_stride_s", "feat_stride_y", "feat_dtype", "mean", "var", "tau",
                     "lag_corr", "feat_mean", "feat_var"):
            setattr(f, name, getattr(s, name))
        f.flags = (self.tabl[0].flags & ~_abi.RAMLT_STATS_WG_MASK) | (s.flags & _abi.RAMLT_STATS_WG_MASK)
        return (_abi.RamltFrame * 1)(f)

    def one_call_step(self, tab):
        """The same step through stats_filter_step (accumulators zeroed first)."""
        self.acc.zero_()
        st = self.lib.stats_filter_step(tab, self.ws_ptr, self.ws_bytes, self.sh)
        if st != 0:
            raise RuntimeError(self._abi.last_error())

    def algorithmic_bytes(self):
        return stats_bytes(self.P, self.S, self.feat_bytes) + self.P * FILTER_STEP_BYTES_PER_PX


def stats_launch_of(flags, table=None):
    """Name of the statistics launch size held in a descriptor's flags (bits 4-7), and with
    ``table`` the tuner's median time per candidate for that table's workload."""
    from paper_2402_08273_amd import _abi
    from paper_2402_08273_amd import tune as _tune

    v = (flags & _abi.RAMLT_STATS_WG_MASK) >> _abi.RAMLT_STATS_WG_SHIFT
    name = _tune.stats_launch_name(v) if v else "4 per CU (library default)"
    if table is None:
        return name
    rec = _tune.TuneCache().record(_tune.stats_workload_key(table, _tune.device_arch()))
    ms = {_tune.stats_launch_name(int(k)): t for k, t in (rec or {}).get("ms", {}).items()}
    return {"chosen": name, "tuning_ms": ms}


def hbm_roofline(nbytes, ms, note, traffic=None):
    """Roofline object of an operation bound by HBM: algorithmic bytes over the measured
    time (HIP events around the operation's launches) against 8 TB/s; ``traffic``: the
    measured HBM bytes of the same launches, when a current record exists, and
    ``traffic_gbs`` the rate those bytes move at over the same time (set only with them)."""
    gbs = nbytes / (ms * 1e-3) / 1e9
    r = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic, "algorithmic_bytes": int(nbytes), "covers": note}
    if traffic:
        r["traffic_gbs"] = traffic_gbs(traffic, ms)
    return r


def traffic_gbs(traffic, ms):
    """GB/s of counted HBM bytes over a measured time, or None without a current record."""
    return round(traffic / (ms * 1e-3) / 1e9, 1) if traffic else None


def time_loop(stream, fn, steps):
    """Milliseconds per call of fn() over `steps` calls, HIP events on the launch stream,
    synchronised on both sides."""
    import torch

    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    for _ in range(steps):
        fn()
    t1.record(stream)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps


def stats_roofline(nbytes, ms, traffic, note):
    """Roofline object of a statistics launch: algorithmic bytes over its duration (HIP
    events on the launch stream) against 8 TB/s, and the committed counter bytes."""
    return hbm_roofline(nbytes, ms, note, traffic)


def measure_uhd(steps, warmup, tune=True, traffic_path=TRAFFIC_RECORDS):
    """The 3840x2160, 256 spp, fp16-feature frame with a 15x15 window: fwd+bwd step (the loss
    formed in the forward pass)."""
    import torch

    from paper_2402_08273_amd.tune import schedule_name
    from synth.workloads import N_REGIONS, UHD

    c = SingleChain(UHD.W, UHD.H, UHD.S, UHD.radius, N_REGIONS, UHD.seed, UHD.frame, UHD.fp16_features, tune)
    for _ in range(warmup):
        c.step()
    ms = time_loop(c.stream, c.step, steps)
    ms_fwd = time_loop(c.stream, lambda: (c.stats(), c.forward()), steps)
    ms_stats = time_loop(c.stream, c.stats, steps)
    b = c.algorithmic_bytes()
    sb = stats_bytes(c.P, c.S, c.feat_bytes)
    res = {
        "workload": f"stats+filter fwd+bwd, {UHD.W}x{UHD.H}, {UHD.S} spp, fp32 radiance + fp16 features, "
                    f"{2 * UHD.radius + 1}x{2 * UHD.radius + 1} window, {N_REGIONS}x{N_REGIONS} regions",
        "mpx_s": round(c.P / (ms * 1e-3) / 1e6, 2),
        "ms_per_step": round(ms, 4),
        "fwd_mpx_s": round(c.P / (ms_fwd * 1e-3) / 1e6, 2),
        "algorithmic_bytes": b,
        "hbm_frac": round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "filter_schedule": schedule_name(c.tabl[0].flags),
        "stats_launch": stats_launch_of(c.tabs[0].flags, c.tabs),
        "stats_ms": round(ms_stats, 4),
        "roofline": stats_roofline(sb, ms_stats, measured_traffic(traffic_path, f"stats {UHD.W}x{UHD.H}x{UHD.S} fp16"),
                                   "stats_kernel (the launches of one stats_accumulate call)"),
    }
    del c
    torch.cuda.empty_cache()
    return res


def measure_batch32(steps, warmup, tune=True, traffic_path=TRAFFIC_RECORDS):
    """32 frames of uneven size and spp; each step is one HIP graph replay of one launch
    per operation over the whole batch (stats, filter, zeroing, fused loss seed + adjoint)."""
    import torch

    from paper_2402_08273_amd.batch import FrameBatch, FrameInput
    from paper_2402_08273_amd.tune import schedule_name
    from synth import gpu as sgpu
    from synth import make_lambda
    from synth.workloads import LAMBDA_SEED, MAX_LAG, N_REGIONS, REFERENCE_SPP, batch32, sample_bytes

    specs = batch32()
    lam = torch.from_numpy(make_lambda(N_REGIONS, seed=LAMBDA_SEED)).cuda()
    frames = []
    for sp in specs:
        rad, feat = sgpu.make_frame(sp.W, sp.H, sp.S, seed=sp.seed, frame=sp.frame)
        ref = sgpu.make_reference(sp.W, sp.H, seed=sp.seed + 1000, frame=sp.frame, spp=REFERENCE_SPP)
        frames.append(FrameInput(rad, feat, ref, lam, radius=sp.radius, n_regions=N_REGIONS, max_lag=MAX_LAG))
    b = FrameBatch(frames, loss_in_forward=True)
    if tune:
        b.stats()
        b.tune()
    b.capture(warmup=1)
    for _ in range(warmup):
        b.replay()
    stream = torch.cuda.current_stream()
    ms = time_loop(stream, b.replay, steps)
    ms_stats = time_loop(stream, b.stats, steps)  # the batched statistics launch alone (eager)
    P = sum(sp.W * sp.H for sp in specs)
    nbytes = sum(sample_bytes(sp) + sp.W * sp.H * (23 * 4 + FILTER_STEP_BYTES_PER_PX) for sp in specs)
    sbytes = sum(sample_bytes(sp) + sp.W * sp.H * 23 * 4 for sp in specs)
    res = {
        "workload": "32 frames 256x256..2048x1152, spp {4,16,64,256}, fp32 radiance+features, 11x11 window, "
                    "20x20 regions; stats+filter fwd+bwd as one HIP graph replay per step",
        "frames": len(specs),
        "pixels": P,
        "samples": sum(sp.W * sp.H * sp.S for sp in specs),
        "mpx_s": round(P / (ms * 1e-3) / 1e6, 2),
        "ms_per_step": round(ms, 4),
        "algorithmic_bytes": nbytes,
        "hbm_frac": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "filter_schedule": schedule_name(b.table[0].flags),
        "stats_launch": stats_launch_of(b.table[0].flags, b.table),
        "stats_ms": round(ms_stats, 4),
        "roofline": stats_roofline(sbytes, ms_stats, measured_traffic(traffic_path, "stats batch32"),
                                   "plan_kernel + stats_batched_kernel (the batch's statistics launch)"),
    }
    del b, frames
    torch.cuda.empty_cache()
    return res


def measure_copy_ceiling(steps, mib=4096):
    """The streaming-copy ceiling of this GPU: a device-to-device copy of ``mib`` MiB
    (torch's copy_, a HIP blit kernel), bytes read + written per second."""
    import torch

    n = mib * (1 << 20) // 4
    src = torch.ones(n, device="cuda:0", dtype=torch.float32)
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    for _ in range(3):
        dst.copy_(src)
    ms = time_loop(stream, lambda: dst.copy_(src), max(steps, 10))
    del src, dst
    torch.cuda.empty_cache()
    gbs = 2 * n * 4 / (ms * 1e-3) / 1e9
    return {"copy_gbs": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4), "bytes": 2 * n * 4,
            "ms": round(ms, 4), "how": f"torch copy_ of {mib} MiB on the device (read + write)"}


def measure_small(steps, warmup, tune=True):
    """The 128 x 128, 16 spp frame with a 7 x 7 window, forward only (stats + filter): it
    fits in the caches, so it is reported per call (launch- and latency-bound)."""
    from synth.workloads import N_REGIONS, SMALL

    c = SingleChain(SMALL.W, SMALL.H, SMALL.S, SMALL.radius, N_REGIONS, SMALL.seed, SMALL.frame, False, tune)
    fwd = lambda: (c.stats(), c.forward())  # noqa: E731
    for _ in range(max(warmup, 10)):
        fwd()
    reps = max(steps, 200)
    ms = time_loop(c.stream, fwd, reps)
    ms_stats = time_loop(c.stream, c.stats, reps)
    return {"workload": f"stats+filter fwd, {SMALL.W}x{SMALL.H}, {SMALL.S} spp, fp32 radiance+features, "
                        f"{2 * SMALL.radius + 1}x{2 * SMALL.radius + 1} window, {N_REGIONS}x{N_REGIONS} regions",
            "us_per_call": round(ms * 1e3, 2), "stats_us": round(ms_stats * 1e3, 2),
            "mpx_s": round(c.P / (ms * 1e-3) / 1e6, 2), "calls_timed": reps,
            "note": "two launches per call, back to back on one stream; the 12.4 MB of inputs stay in the caches"}


def measure_leaf_grad(steps, warmup):
    """The autograd form at 1080p / 64 spp: RegionalFilter.apply on radiance that requires
    grad, MSELoss, backward. Autograd materialises dL/dg for every sample (+12 B per sample
    written: 1.59 GB here), which the algorithmic step does not."""
    import torch

    from paper_2402_08273_amd import ops
    from synth import gpu as sgpu
    from synth import make_lambda
    from synth.workloads import HD, LAMBDA_SEED, N_REGIONS, REFERENCE_SPP

    rad, feat = sgpu.make_frame(HD.W, HD.H, HD.S, seed=HD.seed, frame=HD.frame)
    ref = sgpu.make_reference(HD.W, HD.H, seed=HD.seed + 1000, frame=HD.frame, spp=REFERENCE_SPP)
    lam = torch.from_numpy(make_lambda(N_REGIONS, seed=LAMBDA_SEED)).cuda().requires_grad_(True)
    rad.requires_grad_(True)

    def step():
        rad.grad = None
        lam.grad = None
        out = ops.RegionalFilter.apply(rad, feat, lam, HD.radius, N_REGIONS)
        ops.MSELoss.apply(out, ref).backward()

    for _ in range(warmup):
        step()
    ms = time_loop(torch.cuda.current_stream(), step, steps)
    P = HD.W * HD.H
    extra = P * HD.S * 12
    del rad, feat, ref, lam
    torch.cuda.empty_cache()
    return {"workload": "torch autograd: RegionalFilter -> MSELoss -> backward, 1920x1080, 64 spp, 11x11 window",
            "mpx_s": round(P / (ms * 1e-3) / 1e6, 2), "ms_per_step": round(ms, 4),
            "materialised_grad_bytes": extra,
            "note": "the per-sample gradient is written by autograd (expand of G accumulated into radiance.grad); "
                    "the loss seed runs as its own kernel"}


ADAPT_PROPOSALS = 1 << 24
ADAPT_REGION_COUNTS = (20 * 20, 20 * 20 * 50 * 50)  # the 2-D grid N_top^2; the 4-D grid N_top^2 N_bottom^2


def measure_adapt(steps, warmup, cpu=True, traffic_path=TRAFFIC_RECORDS):
    """region_adapt on 16 M proposals per batch (seeded stream of synth.proposals), for the
    paper's 2-D grid (400 regions) and 4-D grid (10^6 regions); one step = one batch.
    Algorithmic bytes: the proposals (region int32 + alpha float32 = 8 B each) and the
    per-region state read and written (lambda, A_k: 2 x 8 B, i_k, n_k: 2 x 4 B; plus the
    float lambda written: 52 B per region)."""
    import torch

    from paper_2402_08273_amd.ops import RegionAdapter
    from synth.proposals import make_proposals

    out = {"workload": f"Algorithm 1 adaptation, {ADAPT_PROPOSALS} proposals per batch, L = 10, "
                       "gamma_max 1, gamma_scale 5, alpha* 0.5", "proposals": ADAPT_PROPOSALS, "grids": []}
    n = ADAPT_PROPOSALS
    stream = torch.cuda.current_stream()
    for m in ADAPT_REGION_COUNTS:
        region, alpha = make_proposals(n, m, seed=3)
        rd = torch.from_numpy(region).cuda()
        ad_ = torch.from_numpy(alpha).cuda()
        ad = RegionAdapter(m)
        for _ in range(warmup):
            ad.step(rd, ad_)
        ms = time_loop(stream, lambda: ad.step(rd, ad_), steps)
        nbytes = n * 8 + m * 52
        gbs = nbytes / (ms * 1e-3) / 1e9
        out["grids"].append({"regions": m, "ms_per_batch": round(ms, 4),
                             "mproposals_s": round(n / (ms * 1e-3) / 1e6, 1), "algorithmic_bytes": nbytes,
                             "achieved_gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                             "roofline": hbm_roofline(nbytes, ms, "all kernels of one region_adapt call",
                                                      measured_traffic(traffic_path, f"region_adapt 16M {m}")
                                                      if n == 1 << 24 else None)})
        del rd, ad_, ad
    if cpu:
        out["cpu_baseline"] = adapt_cpu_baseline()
    torch.cuda.empty_cache()
    return out


def adapt_cpu_baseline(n=300_000, m=400):
    """The sequential oracle (one proposal at a time, as the algorithm is written) on a
    bounded sample of the same stream, on one host thread."""
    from oracle import region_adapt as ora
    from synth.proposals import make_proposals

    region, alpha = make_proposals(n, m, seed=3)
    st = ora.initial_state(m)
    t0 = time.perf_counter()
    ora.adapt(st, region, alpha)
    dt = time.perf_counter() - t0
    return {"value": round(n / dt / 1e6, 4), "unit": "Mproposals/s", "cores": 1, "kind": "oracle",
            "sample": f"the first {n} proposals of the 400-region stream, {dt:.2f} s"}


def measure_perturb(steps, warmup, cpu=True):
    """Direction perturbation (truncated-normal polar angle, sigma from each proposal's
    region) on 16 M proposals per batch, for 400 and 10^6 regions. Algorithmic bytes per
    proposal: region 4 + omega 12 + (u, v) 8 read, omega' 12 + theta' 4 written = 40 B
    (plus the lambda table, 8 B per region)."""
    import torch

    from paper_2402_08273_amd import ops
    from synth.directions import make_lambda_table, make_perturb_inputs

    n = ADAPT_PROPOSALS
    stream = torch.cuda.current_stream()
    out = {"workload": f"direction perturbation, {n} proposals per batch, sigma_k = sqrt(exp(lambda_k))",
           "proposals": n, "grids": []}
    for m in ADAPT_REGION_COUNTS:
        lam = torch.from_numpy(make_lambda_table(m, seed=5)).cuda()
        region, omega, uv = (torch.from_numpy(a).cuda() for a in make_perturb_inputs(n, m, seed=6))
        fn = lambda: ops.perturb_directions(lam, region, omega, uv, theta=True)
        for _ in range(warmup):
            fn()
        ms = time_loop(stream, fn, steps)
        nbytes = n * 40 + m * 8
        gbs = nbytes / (ms * 1e-3) / 1e9
        out["grids"].append({"regions": m, "ms_per_batch": round(ms, 4),
                             "gproposals_s": round(n / (ms * 1e-3) / 1e9, 2), "algorithmic_bytes": nbytes,
                             "achieved_gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                             "roofline": hbm_roofline(nbytes, ms, "scale_kernel + perturb_kernel",
                                                      measured_traffic(TRAFFIC_RECORDS, f"perturb 16M {m}")),
                             "valu_roofline": valu_roofline(
                                 measured_traffic(TRAFFIC_RECORDS, f"perturb 16M {m}", "valu_insts"), ms,
                                 "perturb_kernel (VALU issue), over the time of scale_kernel + perturb_kernel")})
        del lam, region, omega, uv
    if cpu:
        out["cpu_baseline"] = perturb_cpu_baseline()
    torch.cuda.empty_cache()
    return out


def perturb_cpu_baseline(n=2_000_000, m=400):
    """The oracle (vectorised NumPy/SciPy, float64) on a bounded sample of the 400-region
    stream, on one host thread."""
    from oracle import direction_sampler as ods
    from synth.directions import make_lambda_table, make_perturb_inputs

    lam = make_lambda_table(m, seed=5)
    region, omega, uv = make_perturb_inputs(n, m, seed=6)
    t0 = time.perf_counter()
    ods.perturb_directions(lam, region, omega, uv)
    dt = time.perf_counter() - t0
    return {"value": round(n / dt / 1e6, 3), "unit": "Mproposals/s", "cores": 1, "kind": "oracle",
            "sample": f"the first {n} proposals of the 400-region stream, {dt:.2f} s"}


LENS_CHAINS = 1 << 24
LENS_CAMERA = (1920, 1080, 0.6, 20)   # luminance W, H; tan of half the horizontal field of view; grid N


def measure_lens(steps, warmup, cpu=True):
    """Screen-space chains under the regional adaptive lens perturbation on a 1920x1080
    luminance image, 20x20 regions, 16 M chains: one Metropolis step per chain
    (lens_chain_step), and the closed loop (step, then region_adapt of its (region, alpha)
    stream). The chains carry the luminance and the index of their pixel between steps.
    Algorithmic bytes per chain of the step: omega 12 + noise 12 + carried luminance 4 +
    carried pixel 4 read, region 4 + alpha 4 + carried luminance 4 written, the luminance at
    the proposal 4, omega 12 + pixel 4 written on acceptance (times the batch's mean alpha).

    The steps alone run with a fixed seeded lambda table, so that their time does not depend on
    where the adaptation has just left lambda (with 16 M chains every region closes thousands
    of windows per batch, and lambda swings between its floor, where every proposal stays in
    its pixel and is accepted, and large scales); the closed loop adapts lambda as it goes.

    Order of the launches (the counter records take the timed steps of the first group):
    `warmup` steps alone, `steps` steps alone (timed), `steps` closed-loop steps (timed); then
    the chains regrouped by screen tile (lens_chain_sort) and the same three groups."""
    import torch

    from paper_2402_08273_amd import ops
    from paper_2402_08273_amd.ops import RegionAdapter
    from synth.directions import make_lambda_table
    from synth.lens import make_lens_chains, make_lens_noise, make_luminance

    W, H, tx, N = LENS_CAMERA
    n = LENS_CHAINS
    stream = torch.cuda.current_stream()
    L = torch.from_numpy(make_luminance(W, H, seed=5)).cuda()
    om = torch.from_numpy(make_lens_chains(n, W, H, tx, seed=8)).cuda()
    noise = torch.from_numpy(make_lens_noise(n, seed=9)).cuda()
    ad = RegionAdapter(N * N, L=10)
    dens = torch.full((n,), -1.0, dtype=torch.float32, device=om.device)   # carried luminance
    pix = torch.full((n,), -2, dtype=torch.int32, device=om.device)       # carried pixel
    last = {}

    lam_fixed = torch.from_numpy(make_lambda_table(N * N, seed=7)).cuda()

    def timed(o, nz, d, px):
        def step():
            last["ra"] = ops.lens_chain_step(L, tx, lam_fixed, N, o, nz, density=d, pixel=px)

        def loop():
            last["ra"] = ops.lens_chain_step(L, tx, ad.lam, N, o, nz, density=d, pixel=px)
            ad.step(*last["ra"])

        for _ in range(warmup):
            step()
        ms = time_loop(stream, step, steps)
        region, alpha = last["ra"]
        ok = region >= 0
        acc = float(alpha[ok].double().mean())
        return ms, time_loop(stream, loop, steps), acc

    ms, ms_loop, acc = timed(om, noise, dens, pix)
    nbytes = int(n * (48 + 16 * acc))
    gbs = nbytes / (ms * 1e-3) / 1e9
    # the same chains regrouped by screen tile (lens_chain_sort, 48 B per chain: omega read
    # twice, density read; omega, density and the old index written), then stepped with their
    # noise and carried pixels regrouped the same way
    ms_sort = time_loop(stream, lambda: ops.lens_chain_sort(om, W, H, tx, density=dens), steps)
    om_s, dens_s, perm = ops.lens_chain_sort(om, W, H, tx, density=dens)
    noise_s = noise[perm.long()].contiguous()
    pix_s = pix[perm.long()].contiguous()
    ms_s, ms_loop_s, acc_s = timed(om_s, noise_s, dens_s, pix_s)
    nbytes_s = int(n * (48 + 16 * acc_s))
    out = {"workload": f"lens-perturbation chains, {n} chains, {W}x{H} luminance, {N}x{N} regions, "
                       f"tan(fov/2) = {tx}; steps alone with a fixed seeded lambda table, the adaptive step "
                       f"with region_adapt's lambda",
           "chains": n, "ms_per_step": round(ms, 4), "gchains_s": round(n / (ms * 1e-3) / 1e9, 2),
           "ms_per_adaptive_step": round(ms_loop, 4), "mean_alpha": round(acc, 4), "algorithmic_bytes": nbytes,
           "achieved_gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
           "roofline": hbm_roofline(nbytes, ms, "scale_kernel + lens_step_kernel",
                                    measured_traffic(TRAFFIC_RECORDS, "lens step 16M")),
           "valu_roofline": valu_roofline(measured_traffic(TRAFFIC_RECORDS, "lens step 16M", "valu_insts"), ms,
                                          "lens_step_kernel (VALU issue), over the time of scale_kernel + "
                                          "lens_step_kernel"),
           "tile_order": {"note": "the chains regrouped by 256x256-pixel screen tile (lens_chain_sort)",
                          "ms_per_step": round(ms_s, 4), "ms_per_adaptive_step": round(ms_loop_s, 4),
                          "mean_alpha": round(acc_s, 4),
                          "hbm_frac": round(nbytes_s / (ms_s * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                          "traffic": measured_traffic(TRAFFIC_RECORDS, "lens step 16M tile order"),
                          "traffic_gbs": traffic_gbs(measured_traffic(TRAFFIC_RECORDS, "lens step 16M tile order"),
                                                     ms_s),
                          "valu_roofline": valu_roofline(
                              measured_traffic(TRAFFIC_RECORDS, "lens step 16M tile order", "valu_insts"), ms_s,
                              "lens_step_kernel (VALU issue), over the time of scale_kernel + lens_step_kernel"),
                          "sort_ms": round(ms_sort, 4), "sort_gbs": round(n * 48 / (ms_sort * 1e-3) / 1e9, 1),
                          "ms_per_step_sorting_every_16": round(ms_s + ms_sort / 16, 4)}}
    del L, om, noise, ad, last, dens, pix, om_s, dens_s, perm, noise_s, pix_s, lam_fixed
    if cpu:
        out["cpu_baseline"] = lens_cpu_baseline()
    torch.cuda.empty_cache()
    return out


def lens_cpu_baseline(n=2_000_000):
    """The oracle step (NumPy/SciPy) on a bounded sample of the chains, on one host thread."""
    import numpy as np

    from oracle import lens_chain as olc
    from synth.lens import make_lens_chains, make_lens_noise, make_luminance

    W, H, tx, N = LENS_CAMERA
    L = make_luminance(W, H, seed=5)
    om = make_lens_chains(n, W, H, tx, seed=8)
    noise = make_lens_noise(n, seed=9)
    lam = np.ones(N * N)
    t0 = time.perf_counter()
    olc.step(L, tx, lam, N, om, noise)
    dt = time.perf_counter() - t0
    return {"value": round(n / dt / 1e6, 3), "unit": "Mchains/s", "cores": 1, "kind": "oracle",
            "sample": f"one step of {n} chains (lambda = 1 everywhere), {dt:.2f} s"}


def measure_rrmse(steps, warmup, cpu=True):
    """rRMSE map and image value of a rendered image against its reference at 1920x1080
    and 3840x2160 (synth.images). Algorithmic bytes per pixel: both images read (24 B),
    the map written (4 B)."""
    import torch

    from paper_2402_08273_amd import ops
    from synth.images import make_image_pair

    stream = torch.cuda.current_stream()
    out = {"workload": "rRMSE map + image rRMSE, eps 1e-2", "images": []}
    for W, H in ((1920, 1080), (3840, 2160)):
        I, R = (torch.from_numpy(a).cuda() for a in make_image_pair(W, H, seed=7))
        fn = lambda: ops.rrmse(I, R)
        for _ in range(warmup):
            fn()
        ms = time_loop(stream, fn, steps)
        nbytes = W * H * 28
        gbs = nbytes / (ms * 1e-3) / 1e9
        out["images"].append({"W": W, "H": H, "ms": round(ms, 4), "mpx_s": round(W * H / (ms * 1e-3) / 1e6, 1),
                              "algorithmic_bytes": nbytes, "achieved_gbs": round(gbs, 1),
                              "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                              "roofline": hbm_roofline(nbytes, ms, "rel_error_kernel + finalize",
                                                       measured_traffic(TRAFFIC_RECORDS, f"rrmse {W}x{H}"))})
        del I, R
    if cpu:
        from oracle import rrmse as orr

        I, R = make_image_pair(1920, 1080, seed=7)
        t0 = time.perf_counter()
        orr.rrmse(I, R)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(1920 * 1080 / dt / 1e6, 2), "unit": "Mpixel/s", "cores": 1,
                               "kind": "oracle", "sample": f"the 1920x1080 pair, {dt:.3f} s"}
    torch.cuda.empty_cache()
    return out


def _grow_quadtree(wl, device="cuda"):
    """The forest of a quadtree workload grown over its refinement rounds on the device
    (lookups with visit counting, then a refinement that hands lambda and n_k / 4 to the
    children), and the timed lookup batch."""
    import torch

    from paper_2402_08273_amd.ops import Quadtree, RegionAdapter
    from synth.points import make_points

    R = wl["n_roots"]
    t = Quadtree(R, wl["capacity"], device)
    ad = RegionAdapter(wl["capacity"], device=device)
    root, x, y = make_points(wl["grow_points"], R, seed=wl["seed"], batch=0)
    dev = lambda a: torch.from_numpy(a).to(device)
    g = (dev(x), dev(y), None if R == 1 else dev(root))
    for _ in range(wl["rounds"]):
        t.lookup(*g)
        t.refine(wl["m_split"], ad)
    del g
    root, x, y = make_points(wl["lookup_points"], R, seed=wl["seed"], batch=1)
    batch = (dev(x), dev(y), None if R == 1 else dev(root))
    return t, ad, batch


def measure_quadtree(steps, warmup, cpu=True):
    """Quadtree partitions (2-D: one tree; 4-D: a tree per cell of the 20 x 20 screen grid),
    grown with M_split = 5000 after batches of 10^7 lookups: the lookup of 16 M points with
    visit counting (one step = one batch; algorithmic bytes = x, y (and the root for 4-D)
    read + the leaf written: 12 or 16 B per point; the node table is LDS/L2 resident) and one
    refinement pass on the counts of that batch, state inheritance included."""
    import torch

    from synth.workloads import QUADTREE_2D, QUADTREE_4D

    stream = torch.cuda.current_stream()
    out = {"workload": "quadtree lookup of 16 M points with visit counting, and one refinement pass "
                       "(M_split 5000) on their counts", "trees": []}
    for name, wl in (("2d", QUADTREE_2D), ("4d", QUADTREE_4D)):
        t, ad, (x, y, root) = _grow_quadtree(wl)
        n = x.numel()
        leaf = torch.empty(n, device=x.device, dtype=torch.int32)
        fn = lambda: t.lookup(x, y, root, out=leaf)
        for _ in range(warmup):
            fn()
        nodes = t.n_nodes
        ms = time_loop(stream, fn, steps)
        ms_nc = time_loop(stream, lambda: t.lookup(x, y, root, count=False, out=leaf), steps)
        bpp = 12 if root is None else 16
        gbs = n * bpp / (ms * 1e-3) / 1e9
        # one refinement on the counts of one batch: restore the same tree before each pass
        t.visits.zero_()
        fn()
        snap = [a.clone() for a in (t.child, t.depth, t.visits, t.n_nodes_dev, ad.lam, ad.acc, ad.visits,
                                    ad.updates, ad.lam_f32)]
        live = (t.child, t.depth, t.visits, t.n_nodes_dev, ad.lam, ad.acc, ad.visits, ad.updates, ad.lam_f32)
        times = []
        for rep in range(max(3, steps)):
            for a, b in zip(live, snap):
                a.copy_(b)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            t.refine(wl["m_split"], ad)
            e1.record(stream)
            times.append((e0, e1))
        torch.cuda.synchronize()
        rms = sorted(a.elapsed_time(b) for a, b in times)[len(times) // 2]
        depth = int(t.depth[:t.n_nodes].max())
        out["trees"].append({"partition": name, "roots": wl["n_roots"], "nodes": nodes, "max_depth": depth,
                             "splits_in_timed_refine": (t.n_nodes - nodes) // 4,
                             "lookup_ms": round(ms, 4), "glookups_s": round(n / (ms * 1e-3) / 1e9, 2),
                             "lookup_nocount_ms": round(ms_nc, 4),
                             "bytes_per_point": bpp, "achieved_gbs": round(gbs, 1),
                             "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "refine_ms": round(rms, 4),
                             "roofline": hbm_roofline(n * bpp, ms, "lookup_kernel (one launch)",
                                                      measured_traffic(TRAFFIC_RECORDS, f"quadtree lookup 16M {name}")),
                             "valu_roofline": valu_roofline(
                                 measured_traffic(TRAFFIC_RECORDS, f"quadtree lookup 16M {name}", "valu_insts"), ms,
                                 "lookup_kernel (VALU issue)")})
        del t, ad, x, y, root, leaf, snap, live
    if cpu:
        out["cpu_baseline"] = quadtree_cpu_baseline()
    torch.cuda.empty_cache()
    return out


def quadtree_cpu_baseline(n=2_000_000):
    """The oracle's vectorised lookup (every point descends one level per step) on the 2-D
    forest grown by the oracle itself from the first 10^6 growth points, timed on a bounded
    sample of the timed batch, on one host thread."""
    from oracle import quadtree as oqt
    from synth.points import make_points
    from synth.workloads import QUADTREE_2D as wl

    f = oqt.Forest(1, wl["capacity"])
    _, gx, gy = make_points(1_000_000, 1, seed=wl["seed"], batch=0)
    for _ in range(wl["rounds"]):
        f.lookup_many(None, gx, gy)
        f.refine(wl["m_split"] // 10)
    _, x, y = make_points(n, 1, seed=wl["seed"], batch=1)
    t0 = time.perf_counter()
    f.lookup_many(None, x, y)
    dt = time.perf_counter() - t0
    return {"value": round(n / dt / 1e6, 3), "unit": "Mlookups/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} points on a {len(f.nodes)}-node tree (10^6 growth points per refinement, "
                      f"M_split 500), {dt:.2f} s"}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU. The multi-GPU form of this path (row bands with an r-row "
              "halo, one all-reduce of dL/dlambda; frames of a batch spread over GPUs) is a design "
              "only; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return

    import numpy as np
    import torch

    from paper_2402_08273_amd.tune import schedule_name
    from synth.workloads import HD, MAX_LAG

    torch.cuda.set_device(0)
    if args.only:
        if args.only == "adapt":
            print(json.dumps(measure_adapt(args.steps, args.warmup, cpu=not args.no_cpu_baseline)), flush=True)
            return
        if args.only == "rrmse":
            print(json.dumps(measure_rrmse(args.steps, args.warmup, cpu=not args.no_cpu_baseline)), flush=True)
            return
        if args.only == "perturb":
            print(json.dumps(measure_perturb(args.steps, args.warmup, cpu=not args.no_cpu_baseline)), flush=True)
            return
        if args.only == "lens":
            print(json.dumps(measure_lens(args.steps, args.warmup, cpu=not args.no_cpu_baseline)), flush=True)
            return
        if args.only == "small":
            print(json.dumps(measure_small(args.steps, args.warmup, not args.no_tune)), flush=True)
            return
        if args.only == "leaf_grad":
            print(json.dumps(measure_leaf_grad(args.steps, args.warmup)), flush=True)
            return
        if args.only == "copy":
            print(json.dumps(measure_copy_ceiling(args.steps)), flush=True)
            return
        if args.only == "quadtree":
            print(json.dumps(measure_quadtree(args.steps, args.warmup, cpu=not args.no_cpu_baseline)), flush=True)
            return
        fn = measure_batch32 if args.only == "batched" else measure_uhd
        print(json.dumps(fn(args.steps, args.warmup, not args.no_tune)), flush=True)
        return
    W, H, S, r, N = args.width, args.height, args.spp, args.radius, args.regions
    c = SingleChain(W, H, S, r, N, HD.seed, HD.frame, tune=not args.no_tune)
    P = c.P

    for _ in range(args.warmup):
        c.step()
    torch.cuda.synchronize()

    # ---- timed region: K whole steps; per-launch stats/forward/adjoint durations from HIP
    # events recorded on the launch stream inside the same region, around the launches of
    # every MARK_EVERY-th step (an event between launches costs a few microseconds)
    marked = list(range(0, args.steps, MARK_EVERY))
    marks = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in marked]
    step_no = iter(range(args.steps))
    mark_of = dict(zip(marked, marks))
    ms_step = time_loop(c.stream, lambda: c.step(mark_of.get(next(step_no))), args.steps)
    stats_ms = float(np.mean([m[0].elapsed_time(m[1]) for m in marks]))
    fwd_ms = float(np.mean([m[0].elapsed_time(m[2]) for m in marks]))
    adj_ms = float(np.mean([m[2].elapsed_time(m[3]) for m in marks]))
    # whole-step durations, one pair of events around each step: the median
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    for e in ev:
        e[0].record(c.stream)
        c.step()
        e[1].record(c.stream)
    torch.cuda.synchronize()
    step_ms_median = float(np.median([e[0].elapsed_time(e[1]) for e in ev]))

    # the other forms of the step: plain forward + adjoint with the seed fused; separate
    # loss_seed kernel writing U; forward only (stats + filter)
    fused_ms = time_loop(c.stream, lambda: c.step(form="fused"), args.steps)
    unfused_ms = time_loop(c.stream, lambda: c.step(form="unfused"), args.steps)
    fwd_only_ms = time_loop(c.stream, lambda: (c.stats(), c.forward()), args.steps)
    tab1 = c.one_call_table()
    one_call_ms = time_loop(c.stream, lambda: c.one_call_step(tab1), args.steps)

    sb = stats_bytes(P, S)
    achieved = sb / (stats_ms * 1e-3) / 1e9
    traffic = measured_traffic(args.traffic, f"stats {W}x{H}x{S}") if (W, H, S) == (HD.W, HD.H, HD.S) else None
    step_bytes = c.algorithmic_bytes()

    result = {
        "metric": "Mpixel/s filtered (fwd, fwd+bwd) at 1080p 64spp; % of HBM roofline",
        "value": round(P / (ms_step * 1e-3) / 1e6, 2),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 in, f64 stats accumulate, f32 filter",
        "data": "synthetic (seeded scene: ramp + hard edge + disc, per-pixel noise U[0.02,0.5], 0.1% lognormal "
                "fireflies; 4096-spp seeded reference)",
        "config": {"workload": f"stats+filter fwd+bwd, {W}x{H}, {S} spp, fp32 radiance+features, "
                               f"{2 * r + 1}x{2 * r + 1} window, {N}x{N} regions",
                   "width": W, "height": H, "spp": S, "radius": r, "regions": N, "max_lag": MAX_LAG},
        "ms_per_step_median": round(step_ms_median, 4),
        "step_form": "loss in the forward pass (stats -> filter with seed, loss, dL/dlambda -> radiance adjoint)",
        "fwd_mpx_s": round(P / (fwd_only_ms * 1e-3) / 1e6, 2),
        "fused_adjoint_fwd_bwd_mpx_s": round(P / (fused_ms * 1e-3) / 1e6, 2),
        "unfused_fwd_bwd_mpx_s": round(P / (unfused_ms * 1e-3) / 1e6, 2),
        "one_call_fwd_bwd_mpx_s": round(P / (one_call_ms * 1e-3) / 1e6, 2),
        "fwd_ms": round(fwd_only_ms, 4),
        "stats_ms": round(stats_ms, 4),
        "filter_forward_with_loss_ms": round(fwd_ms - stats_ms, 4),
        "radiance_adjoint_ms": round(adj_ms, 4),
        "filter_schedule": schedule_name(c.tabl[0].flags),
        "filter_schedule_fwd_only": schedule_name(c.tabf[0].flags),
        "stats_launch": stats_launch_of(c.tabs[0].flags, c.tabs),
        "roofline": {
            "kernel": "stats_accumulate",
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "traffic_gbs": traffic_gbs(traffic, stats_ms),
            "algorithmic_bytes": sb,
        },
        # whole step: the statistics pass, the forward with the loss (mean, reference read;
        # out, U written) and the radiance adjoint (U read, G written), over the step's time,
        # against the 0.70 of 8 TB/s the step is meant to reach
        "step_roofline": {
            "covers": "whole step (all kernels)",
            "bound": "hbm",
            "achieved": round(step_bytes / (ms_step * 1e-3) / 1e9, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "target_frac": 0.70,
            "algorithmic_bytes": step_bytes,
        },
        "step_algorithmic_gbs": round(step_bytes / (ms_step * 1e-3) / 1e9, 1),
        "step_hbm_frac": round(step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
    }

    one_thread = None
    if not args.no_cpu_baseline:
        one_thread = cpu_baseline(c.rad, c.feat, c.ref, c.lam, W, H, S, r, N, args.cpu_rows)
    del c
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        par = cpu_baseline_parallel(W, H, S, r, N, HD.seed, HD.frame)
        par["single_thread"] = {k: one_thread[k] for k in ("value", "unit", "sample", "seconds")}
        result["cpu_baseline"] = par
    result["copy_ceiling"] = measure_copy_ceiling(args.steps)
    result["roofline"]["frac_of_copy_ceiling"] = round(achieved / result["copy_ceiling"]["copy_gbs"], 4)

    if not args.no_extra:
        print("measuring the small frame, the autograd form, the 32-frame batch and the 4K frame", file=sys.stderr,
              flush=True)
        result["small"] = measure_small(args.steps, args.warmup, not args.no_tune)
        result["leaf_grad"] = measure_leaf_grad(args.steps, args.warmup)
        result["batched"] = measure_batch32(args.steps, args.warmup, not args.no_tune)
        result["uhd"] = measure_uhd(args.steps, args.warmup, not args.no_tune)
        result["adapt"] = measure_adapt(args.steps, args.warmup, cpu=not args.no_cpu_baseline)
        result["quadtree"] = measure_quadtree(args.steps, args.warmup, cpu=not args.no_cpu_baseline)
        result["perturb"] = measure_perturb(args.steps, args.warmup, cpu=not args.no_cpu_baseline)
        result["rrmse"] = measure_rrmse(args.steps, args.warmup, cpu=not args.no_cpu_baseline)
        result["lens"] = measure_lens(args.steps, args.warmup, cpu=not args.no_cpu_baseline)

    print(json.dumps(result), flush=True)


def _oracle_chain(rad_b, feat_b, ref_b, lam_h, S, r, N, W, H, y0=0):
    import oracle

    crop = dict(origin=(0, y0), image_size=(W, H))
    st = oracle.stats_accumulate(rad_b, feat_b, 8)
    out, _ = oracle.filter_forward(st["mean"], lam_h, N, r, -30.0, **crop)
    _, U = oracle.mse_loss_seed(out, ref_b, count=3 * W * H)
    oracle.filter_backward(U, st["mean"], out, lam_h, N, r, -30.0, S, **crop)


def cpu_baseline(rad, feat, ref, lam, W, H, S, r, N, rows, target_s=15.0):
    """The FP64 oracle, as it stands, on a band of rows of the same frame (same chain:
    stats -> filter -> loss seed -> adjoint, with the frame's regions), timed on the host.
    Rate in Mpixel/s. The band height is chosen from two probes (8 and 24 rows: their
    difference removes the fixed cost of a call) so the timed run takes about target_s."""
    lam_h = lam.cpu().numpy()

    def band(n):
        sl = slice(0, n)
        return rad[:, :, sl].cpu().numpy(), feat[:, :, sl].cpu().numpy(), ref[:, sl].cpu().numpy()

    if not rows:
        times = []
        for probe in (min(8, H), min(24, H)):
            t0 = time.perf_counter()
            _oracle_chain(*band(probe), lam_h, S, r, N, W, H)
            times.append((probe, time.perf_counter() - t0))
        (p0, t0_), (p1, t1_) = times
        per_row = (t1_ - t0_) / (p1 - p0) if p1 > p0 and t1_ > t0_ else t1_ / p1
        rows = int(max(p1, min(H, target_s / max(per_row, 1e-6))))
    data = band(rows)
    t0 = time.perf_counter()
    _oracle_chain(*data, lam_h, S, r, N, W, H)
    dt = time.perf_counter() - t0
    px = W * rows
    return {
        "value": round(px / dt / 1e6, 5),
        "unit": "Mpixel/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"rows 0..{rows - 1} of the {W}x{H} frame ({px} px, {S} spp, features), full "
                  f"stats+filter+loss+adjoint chain in numpy fp64 on one thread, {dt:.2f} s",
        "seconds": round(dt, 3),
    }


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or "unknown"."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores(cap=16):
    """Threads the CPU baseline may use: the CPU share of this process (at most ``cap``, the
    share of one GPU on the GPU hosts)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, cap))


def _band_worker(W, H, S, r, N, seed, frame, y0, y1, ref_spp, barrier, queue):
    """One band of rows [y0, y1) of the frame: its inputs with a 2r-row halo on each side
    (generated here, untimed), then the oracle chain on that crop, timed between two
    barriers shared with the other bands."""
    import numpy as np

    from synth import numpy_gen
    from synth.workloads import LAMBDA_SEED

    a, b = max(0, y0 - 2 * r), min(H, y1 + 2 * r)
    rad, feat = numpy_gen.make_frame(W, H, S, seed, frame, rows=(a, b))
    ref = numpy_gen.make_reference(W, H, seed + 1000, frame, spp=ref_spp, rows=(a, b))
    lam = numpy_gen.make_lambda(N, seed=LAMBDA_SEED).astype(np.float64)
    barrier.wait()
    t0 = time.monotonic()
    _oracle_chain(rad, feat, ref, lam, S, r, N, W, H, y0=a)
    queue.put((y0, y1, t0, time.monotonic()))


def cpu_baseline_parallel(W, H, S, r, N, seed, frame, cores=None, ref_spp=64, timeout=600):
    """The FP64 oracle, as it stands, band-parallel over the host cores: the frame's rows
    split into one band per core, each band (plus the 2r-row halo its filter and adjoint
    read) run through the whole chain (stats -> filter -> loss seed -> adjoint) by one
    process, all bands timed together (wall clock from the first start to the last end).
    The bands' inputs come from the NumPy twin of the input recipe (the reference from
    ``ref_spp`` samples: the oracle's work does not depend on its values)."""
    import multiprocessing as mp

    cores = cores or host_cores()
    ctx = mp.get_context("spawn")  # fresh interpreters: nothing of this process's GPU state
    barrier = ctx.Barrier(cores)
    queue = ctx.Queue()
    edges = [round(i * H / cores) for i in range(cores + 1)]
    procs = [ctx.Process(target=_band_worker, args=(W, H, S, r, N, seed, frame, edges[i], edges[i + 1], ref_spp,
                                                    barrier, queue), daemon=True) for i in range(cores)]
    for p in procs:
        p.start()
    import queue as _q

    got = []
    t_end = time.monotonic() + timeout
    try:
        while len(got) < cores:
            try:
                got.append(queue.get(timeout=2))
            except _q.Empty:
                dead = [p.exitcode for p in procs if p.exitcode not in (None, 0)]
                if dead or time.monotonic() > t_end:
                    raise RuntimeError(f"CPU baseline band failed (exit codes {dead})")
    finally:
        for p in procs:
            p.join(timeout=30)
            if p.is_alive():
                p.kill()
    wall = max(g[3] for g in got) - min(g[2] for g in got)
    return {
        "value": round(W * H / wall / 1e6, 5),
        "unit": "Mpixel/s",
        "cores": cores,
        "cpu": cpu_model(),
        "kind": "oracle",
        "sample": f"the whole {W}x{H} frame ({W * H} px, {S} spp, features) in {cores} row bands, one process "
                  f"each, full stats+filter+loss+adjoint chain in numpy fp64, {wall:.2f} s wall",
        "seconds": round(wall, 3),
    }


if __name__ == "__main__":
    main()
