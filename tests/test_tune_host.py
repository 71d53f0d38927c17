"""Host logic of the autotuner: the cache round trip, workload keys, schedule names."""

import json

from paper_2402_08273_amd import _abi
from paper_2402_08273_amd import tune


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    c = tune.TuneCache(path)
    assert c.get("k") is None
    c.put("k", _abi.RAMLT_TILE_64X8, {_abi.RAMLT_TILE_32X8: 0.2, _abi.RAMLT_TILE_64X8: 0.1})
    again = tune.TuneCache(path)
    assert again.get("k") == _abi.RAMLT_TILE_64X8
    rec = json.load(open(path))["k"]
    assert rec["name"] == "64x8/separable" and set(rec["ms"]) == {"1", "3"}


def test_corrupt_cache_is_ignored(tmp_path):
    path = tmp_path / "tune.json"
    path.write_text("{not json")
    assert tune.TuneCache(str(path)).get("x") is None


def test_keys_and_names():
    a, b = _abi.RamltFrame(), _abi.RamltFrame()
    a.W, a.H, a.S, a.radius, a.n_regions = 1920, 1080, 64, 5, 20
    b.W, b.H, b.S, b.radius, b.n_regions = 256, 256, 4, 5, 20
    k1 = tune.workload_key([a, b], "gfx950")
    k2 = tune.workload_key([b, a], "gfx950")
    assert k1 != k2 and k1.startswith("gfx950|1920x1080x64/r5/N20;")
    assert tune.schedule_name(0) == "32x8/separable"
    assert tune.schedule_name(_abi.RAMLT_TILE_32X16 | _abi.RAMLT_SCHED_DIRECT) == "32x16/direct"
    # every candidate is a valid flags value and they are distinct
    assert len(set(tune.CANDIDATES)) == len(tune.CANDIDATES)
    assert all(c & ~(_abi.RAMLT_TILE_MASK | _abi.RAMLT_SCHED_DIRECT) == 0 for c in tune.CANDIDATES)


def test_stats_keys_and_candidates():
    a = _abi.RamltFrame()
    a.W, a.H, a.S, a.max_lag = 3840, 2160, 256, 8
    a.features, a.feat_dtype = 0x1000, _abi.RAMLT_F16
    b = _abi.RamltFrame.from_buffer_copy(a)
    b.features = None
    assert tune.stats_workload_key([a], "gfx950") == "stats|gfx950|3840x2160x256/f16/L8"
    assert tune.stats_workload_key([b], "gfx950") == "stats|gfx950|3840x2160x256/none/L8"
    b.S = 4  # the lag is clipped to S - 1, as the library clips it
    assert tune.stats_workload_key([b], "gfx950").endswith("/L3")
    # launch sizes fit the 4-bit field, and none is the library default (0)
    assert len(set(tune.STATS_CANDIDATES)) == len(tune.STATS_CANDIDATES)
    assert all(1 <= v <= 15 for v in tune.STATS_CANDIDATES)
    assert _abi.RAMLT_STATS_ONE_LAUNCH in tune.STATS_CANDIDATES
    assert tune.stats_launch_name(15) == "one launch" and tune.stats_launch_name(3) == "3 per CU"
    # the field does not overlap the filter schedule bits or the loss flag
    assert _abi.RAMLT_STATS_WG_MASK & (tune.SCHEDULE_BITS | _abi.RAMLT_LOSS_IN_FORWARD) == 0
