"""The committed counter files belong to the kernels in the tree (CPU only).

bench.py reports `roofline.traffic` (and the backward's) from profiles/*_traffic.json only when the
file's kernel hash equals the hash of the current kernel sources; these checks keep the committed
profiles from going stale silently when a kernel source changes.
"""
import json
import os

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_forward_traffic_file_matches_the_forward_kernel_sources():
    with open(bench.TRAFFIC_FILE) as fh:
        entries = json.load(fh)["entries"]
    hashes = {e["kernel_hash"] for e in entries}
    assert bench.kernel_hash() in hashes
    headline = [e for e in entries if e["kernel_hash"] == bench.kernel_hash()]
    assert any(tuple(e["plan"]) == tuple(bench.HEADLINE_PLAN) for e in headline)
    for e in headline:
        # calibrated counter bytes: within 10% above the algorithmic bytes (halo re-reads), never below
        assert e["algorithmic_bytes_per_launch"] <= e["bytes_per_launch"] <= 1.1 * e["algorithmic_bytes_per_launch"]


def test_backward_traffic_file_matches_the_backward_kernel_sources():
    with open(bench.BWD_TRAFFIC_FILE) as fh:
        tr = json.load(fh)
    assert tr["kernel_hash"] == bench.kernel_hash(bench.BWD_KERNEL_SOURCES)
    assert tr["workload"][:4] == [64, 65536, 50, 15]
    assert tr["algorithmic_bytes_per_launch"] <= tr["bytes_per_launch"] <= 1.1 * tr["algorithmic_bytes_per_launch"]


def test_headline_profile_names_the_current_forward_hash():
    with open(os.path.join(ROOT, "profiles", "ldbp_fwd_64x65536_l50_T15.md")) as fh:
        assert bench.kernel_hash() in fh.read()
    with open(os.path.join(ROOT, "profiles", "ldbp_bwd_64x65536_l50_T15.md")) as fh:
        assert bench.kernel_hash(bench.BWD_KERNEL_SOURCES) in fh.read()
