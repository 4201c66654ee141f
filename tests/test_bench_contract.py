"""The benchmark's host-side contract (CPU only): the single-GPU guard, the
choice of the roofline kernel and its per-launch time, and the stored-traffic
lookup, which must name the kernel's current source."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "single GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def _res(m2l_f, m2l_a, p2p):
    return {"phases_fwd_ms": {"m2l": m2l_f, "p2p": p2p}, "phases_adj_ms": {"m2l": m2l_a, "p2p": 2 * p2p},
            "counts": {"m2l_rank": 116, "v_pairs": 1000, "p2p_pairs": 5000}}


def test_roofline_takes_the_kernel_with_most_time_per_step():
    r = bench.roofline(_res(1.0, 1.4, 0.9), 152, "split_bf16", "none", 1)
    assert r["kernel"] == "k_m2l" and r["bound"] == "mfma"
    assert r["per_launch_ms"] == pytest.approx(1.2)   # mean of the two launches in a step
    assert r["achieved"] == pytest.approx(2 * 116 * 116 * 1000 / 1.2e-3 / 1e12)
    assert r["peak"] == 2500.0 and r["frac"] == pytest.approx(r["achieved"] / 2500.0)
    r = bench.roofline(_res(0.4, 0.5, 2.0), 152, "fp32", "none", 1)
    assert r["kernel"] == "k_p2p" and r["bound"] == "alu" and r["per_launch_ms"] == 2.0
    assert r["achieved"] == pytest.approx(20 * 5000 / 2.0e-3 / 1e12)
    assert r["traffic"] is None   # nothing stored for this workload
    # the near-field roofline is reported beside the M2L's whichever dominates
    q = bench.near_roofline(_res(1.0, 1.4, 0.9), "split_bf16", "none", 1)
    assert q["kernel"] == "k_p2p" and q["per_launch_ms"] == 0.9
    assert q["frac"] == pytest.approx(20 * 5000 / 0.9e-3 / 1e12 / 157.3)


def test_stored_traffic_follows_the_sources():
    # a stored traffic figure is reported only while the kernel's source file
    # is the one the counters were taken with, else null
    recs = [json.loads(l[len("traffic_json: "):]) for l in open(bench.TRAFFIC_FILE) if l.startswith("traffic_json: ")]
    assert recs
    for r in recs:
        t = bench.stored_traffic(r["kernel"], r["precision"], r["workload"], r["n"])
        if r["source_sha256_16"] == bench.source_digest(r["kernel"]):
            assert t == r["bytes_per_launch"] and t > 0
        else:
            assert t is None
