"""Host logic of bench.py (no GPU): the HBM-traffic figure comes from a
committed counter summary only while the hash of its kernel sources matches
the tree, and --gpus above 1 is refused."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_counter_summaries_parse_and_match_their_workload():
    for grp in ("push", "deposit"):
        path = os.path.join(ROOT, "profiles", f"{grp}_c3_counters.txt")
        assert os.path.exists(path)
        kv = dict(l.split(":", 1) for l in open(path) if ":" in l and not l.startswith("#"))
        assert int(kv["particles"]) == bench.WORKLOADS["c3"]["n"]
        assert float(kv["fetch_factor"]) > 0 and float(kv["write_factor"]) > 0
    # a summary for another particle count is not used
    assert bench.counter_traffic("push", "c3", 12345) is None
    # nor one for a workload that has none
    assert bench.counter_traffic("push", "c2", bench.WORKLOADS["c2"]["n"]) is None


def test_traffic_is_null_once_the_kernel_sources_change(monkeypatch):
    n = bench.WORKLOADS["c3"]["n"]
    real = bench.kernel_source_hash
    monkeypatch.setattr(bench, "kernel_source_hash", lambda g: "0" * 64)
    assert bench.counter_traffic("push", "c3", n) is None
    monkeypatch.setattr(bench, "kernel_source_hash", real)
    path = os.path.join(ROOT, "profiles", "push_c3_counters.txt")
    kv = dict(l.split(":", 1) for l in open(path) if ":" in l and not l.startswith("#"))
    if kv["kernel_source_sha256"].strip() == real("push"):
        t = bench.counter_traffic("push", "c3", n)
        assert t is not None and 100 * n < t < 400 * n


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr
