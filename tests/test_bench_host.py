"""Host-side accounting of bench.py (no GPU): algorithmic bytes per stream-collide
launch, the segment count it uses, and the traffic lookup keyed by kernel source."""
import json
import os

import numpy as np

import bench


class _Info:
    def __init__(self, n_active):
        self.n_active = n_active


def test_algorithmic_bytes():
    # 7 FP32 reads + 7 FP32 writes per fluid update, +4 B of 1/tau with Knudsen,
    # and 120 B record + 4 B list entry per visited segment
    # 56 B of populations + 1 B of flags per fluid update, + 4 B of 1/tau with Knudsen
    assert bench.algorithmic_bytes(_Info(256), knudsen=False) == 256 * 57
    assert bench.algorithmic_bytes(_Info(256), knudsen=True) == 256 * 61
    assert bench.metadata_bytes(4) == 4 * 124


def test_traffic_lookup_requires_matching_kernel_source():
    path = os.path.join(bench.ROOT, "profiles", "traffic.json")
    with open(path) as fh:
        d = json.load(fh)
    (workload, entry), = d.items()
    assert bench.traffic_from_profiles(entry["kernel_sha"], workload) == entry["bytes_per_launch"]
    assert bench.traffic_from_profiles("0" * 16, workload) is None
    assert bench.traffic_from_profiles(entry["kernel_sha"], "no such workload") is None


def test_more_than_one_gpu_is_refused():
    import subprocess
    import sys

    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
