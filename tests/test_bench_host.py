"""bench.py on the host: it measures one GPU and refuses more with a message (before any GPU
call), and its byte and traffic bookkeeping matches the workload it names."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    run = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert run.returncode != 0
    assert "one GPU" in run.stderr and run.stdout == ""


def test_statistics_bytes_and_traffic_records():
    P, S = 1920 * 1080, 64
    # every sample read once (3 radiance fp32 + 7 features) and 23 fp32 output planes
    assert bench.stats_bytes(P, S) == P * S * 40 + P * 23 * 4 == 5_499_187_200
    assert bench.stats_bytes(P, S, feat_bytes=2) == P * S * 26 + P * 23 * 4
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    data = json.load(open(path))
    cal = data["copy_calibration"]
    import hashlib

    for rec in data["records"]:
        # scaled counter bytes: FETCH_SIZE and WRITE_SIZE (KiB) times the copy calibration
        scaled = rec["fetch_kib"] * 1024 * cal["fetch_scale"] + rec["write_kib"] * 1024 * cal["write_scale"]
        assert rec["bytes_per_launch"] == int(scaled), rec["key"]
        # a record counts for the kernel sources it was taken on only
        h = hashlib.sha256()
        for src in rec["sources"]:
            h.update(open(os.path.join(ROOT, src), "rb").read())
        same = h.hexdigest()[:16] == rec["sources_sha256_16"]
        assert bench.measured_traffic(path, rec["key"]) == (rec["bytes_per_launch"] if same else None)
    assert bench.measured_traffic(path, "no such workload") is None
    assert bench.measured_traffic("", "stats 1920x1080x64") is None
