"""Autotuner for the launch schedules: the filter's output tile shape (32x8, 32x16, 64x8)
and window schedule (separable rows-then-columns, or the direct (2r+1)^2 gather), and the
statistics pass's launch size (workgroups per compute unit per launch, or one launch).

The schedule is a field of every frame descriptor (``ramlt_frame.flags``); it changes the
launch, not the result beyond fp32 rounding order. The tuner times each candidate on the
caller's own frames on the device (HIP events on the launch stream, forward + adjoint as
one step uses them), keeps the fastest, and remembers it in a JSON cache keyed by the
device architecture and the frame shapes, so later runs with the same shapes skip the
timing. All timing runs through ``libramlt.so``; nothing here computes on the host.

Cache file: ``$RAMLT_TUNE_CACHE`` if set, else ``~/.cache/ramlt/tune.json``.
"""

import ctypes
import json
import os
import threading
from typing import Dict, Iterable, List, Optional, Sequence

import torch

from . import _abi

CANDIDATES = (
    _abi.RAMLT_TILE_32X8,
    _abi.RAMLT_TILE_32X16,
    _abi.RAMLT_TILE_64X8,
    _abi.RAMLT_TILE_32X8 | _abi.RAMLT_SCHED_DIRECT,
)
SCHEDULE_BITS = _abi.RAMLT_TILE_MASK | _abi.RAMLT_SCHED_DIRECT
# statistics launch sizes (workgroups per compute unit per launch; 15 = one launch)
STATS_CANDIDATES = (2, 3, 4, 5, 6, 8, _abi.RAMLT_STATS_ONE_LAUNCH)

_lock = threading.Lock()


def schedule_name(flags: int) -> str:
    w, h = _abi.TILE_SHAPES.get(flags & _abi.RAMLT_TILE_MASK or _abi.RAMLT_TILE_32X8)
    return f"{w}x{h}" + ("/direct" if flags & _abi.RAMLT_SCHED_DIRECT else "/separable")


def cache_path() -> str:
    return os.environ.get("RAMLT_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "ramlt",
                                                              "tune.json")


class TuneCache:
    """A JSON map from workload key to {"schedule": flags, "ms": {flags: milliseconds}}."""

    def __init__(self, path: Optional[str] = None):
        self.path = path or cache_path()
        self._data: Dict[str, dict] = {}
        if os.path.exists(self.path):
            try:
                with open(self.path) as fh:
                    self._data = json.load(fh)
            except (OSError, ValueError):
                self._data = {}

    def get(self, key: str) -> Optional[int]:
        rec = self._data.get(key)
        return None if rec is None else int(rec["schedule"])

    def record(self, key: str) -> Optional[dict]:
        return self._data.get(key)

    def put(self, key: str, schedule: int, timings: Dict[int, float], name: Optional[str] = None):
        self._data[key] = {"schedule": int(schedule), "name": name or schedule_name(schedule),
                           "ms": {str(k): round(v, 5) for k, v in timings.items()}}
        with _lock:
            os.makedirs(os.path.dirname(self.path) or ".", exist_ok=True)
            tmp = self.path + f".{os.getpid()}.tmp"
            with open(tmp, "w") as fh:
                json.dump(self._data, fh, indent=1, sort_keys=True)
            os.replace(tmp, self.path)


def device_arch(device=None) -> str:
    props = torch.cuda.get_device_properties(device or torch.cuda.current_device())
    return getattr(props, "gcnArchName", "unknown").split(":")[0]


def workload_key(descs: Iterable, arch: str) -> str:
    """Key of a list of frame descriptors: architecture + each frame's (W, H, S, radius,
    regions, whether the loss is formed in the forward pass), in order (S matters to the
    adjoint only through its scale, but is kept so a key names one workload)."""
    parts = [f"{d.W}x{d.H}x{d.S}/r{d.radius}/N{d.n_regions}"
             + ("/loss-in-forward" if getattr(d, "flags", 0) & _abi.RAMLT_LOSS_IN_FORWARD else "") for d in descs]
    return arch + "|" + ";".join(parts)


def _median_ms(fn, stream, reps: int, warmup: int) -> float:
    for _ in range(warmup):
        fn()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    torch.cuda.synchronize()
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    times = sorted(a.elapsed_time(b) for a, b in evs)
    return times[len(times) // 2]


def tune_table(table, stream=None, device=None, candidates: Sequence[int] = CANDIDATES, reps: int = 10,
               warmup: int = 3, cache: Optional[TuneCache] = None, force: bool = False,
               zero: Optional[List[torch.Tensor]] = None) -> int:
    """Pick the schedule for the frames of ``table`` (a ctypes array of RamltFrame whose
    buffers are live on the device: mean, lambda, out, grad buffers, reference): times
    filter_forward + filter_backward for every candidate, writes the winner into every
    descriptor's flags and returns it. The adjoint accumulates into grad_lambda and loss:
    pass those tensors in ``zero`` to clear them after timing."""
    device = torch.device(device or torch.cuda.current_device())
    stream = stream or torch.cuda.current_stream(device)
    cache = cache if cache is not None else TuneCache()
    key = workload_key(table, device_arch(device))
    best = None if force else cache.get(key)
    if best is None:
        lib = _abi.load()
        n = len(table)
        old = [d.flags for d in table]
        timings = {}
        for cand in candidates:
            for d in table:
                d.flags = (d.flags & ~SCHEDULE_BITS) | cand
            table_dev, ws_keep, ws_ptr, ws_bytes = _device_state(table, device)

            def step():
                for name in ("filter_forward", "filter_backward"):
                    st = getattr(lib, name)(table, table_dev, n, ws_ptr, ws_bytes, stream.cuda_stream)
                    if st != _abi.RAMLT_OK:
                        raise _abi.RamltError(st, _abi.last_error())

            timings[cand] = _median_ms(step, stream, reps, warmup)
            del ws_keep
        best = min(timings, key=timings.get)
        for d, f in zip(table, old):
            d.flags = f
        cache.put(key, best, timings)
    for d in table:
        d.flags = (d.flags & ~SCHEDULE_BITS) | best
    for t in zero or ():
        t.zero_()
    return best


def _device_state(table, device):
    """Device copy of the table (for batches) and a workspace for the filter operations."""
    n = len(table)
    table_dev = None
    keep = []
    if n > 1:
        raw = bytes(ctypes.string_at(ctypes.addressof(table), ctypes.sizeof(table)))
        t = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(device)
        keep.append(t)
        table_dev = t.data_ptr()
    need = max(_abi.workspace_size(list(table), op) for op in (_abi.OP_FILTER_FORWARD, _abi.OP_FILTER_BACKWARD))
    ws_ptr = None
    if need:
        w = torch.empty(need + 256, device=device, dtype=torch.uint8)
        keep.append(w)
        ws_ptr = (w.data_ptr() + 255) // 256 * 256
    return table_dev, keep, ws_ptr, need


def stats_workload_key(descs: Iterable, arch: str) -> str:
    """Key of the statistics pass over a list of frame descriptors: architecture + each
    frame's (W, H, S, feature dtype or none, maximum lag), in order."""
    parts = []
    for d in descs:
        feat = "none" if not d.features else ("f16" if d.feat_dtype == _abi.RAMLT_F16 else "f32")
        parts.append(f"{d.W}x{d.H}x{d.S}/{feat}/L{min(d.max_lag, d.S - 1)}")
    return "stats|" + arch + "|" + ";".join(parts)


def stats_launch_name(v: int) -> str:
    return "one launch" if v == _abi.RAMLT_STATS_ONE_LAUNCH else f"{v} per CU"


def tune_stats(table, stream=None, device=None, candidates: Sequence[int] = STATS_CANDIDATES, reps: int = 10,
               warmup: int = 3, cache: Optional[TuneCache] = None, force: bool = False, table_dev=None) -> int:
    """Pick the statistics pass's launch size for the frames of ``table`` (a ctypes array of
    RamltFrame whose sample planes and statistics outputs are live on the device; for more
    than one frame ``table_dev`` is the device copy of the table, which is rewritten for each
    candidate): times stats_accumulate for every candidate, writes the winner into bits
    4-7 of every descriptor's flags (the library reads the first) and returns it."""
    device = torch.device(device or torch.cuda.current_device())
    stream = stream or torch.cuda.current_stream(device)
    cache = cache if cache is not None else TuneCache()
    key = stats_workload_key(table, device_arch(device))
    best = None if force else cache.get(key)
    n = len(table)
    if n > 1 and table_dev is None:
        raise ValueError("a batch needs the device copy of its table")

    def put(v):
        for d in table:
            d.flags = (d.flags & ~_abi.RAMLT_STATS_WG_MASK) | (v << _abi.RAMLT_STATS_WG_SHIFT)
        if n > 1:
            raw = bytes(ctypes.string_at(ctypes.addressof(table), ctypes.sizeof(table)))
            table_dev.copy_(torch.frombuffer(bytearray(raw), dtype=torch.uint8))

    if best is None:
        lib = _abi.load()
        need = _abi.workspace_size(list(table), _abi.OP_STATS)
        w = torch.empty(need + 256, device=device, dtype=torch.uint8) if need else None
        ws_ptr = (w.data_ptr() + 255) // 256 * 256 if need else None
        dev_ptr = table_dev.data_ptr() if n > 1 else None
        timings = {}
        for cand in candidates:
            put(cand)

            def run():
                st = lib.stats_accumulate(table, dev_ptr, n, ws_ptr, need, stream.cuda_stream)
                if st != _abi.RAMLT_OK:
                    raise _abi.RamltError(st, _abi.last_error())

            timings[cand] = _median_ms(run, stream, reps, warmup)
        best = min(timings, key=timings.get)
        cache.put(key, best, timings, name=stats_launch_name(best))
    put(best)
    return best


def tuned_schedule(W, H, S, radius, n_regions, device=None, cache: Optional[TuneCache] = None) -> int:
    """The cached schedule of a single frame of this shape, or 0 (library default)."""
    cache = cache if cache is not None else TuneCache()

    class _D:  # the fields workload_key reads
        pass

    d = _D()
    d.W, d.H, d.S, d.radius, d.n_regions = W, H, S, radius, n_regions
    got = cache.get(workload_key([d], device_arch(device)))
    return 0 if got is None else got
