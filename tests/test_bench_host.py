"""Host-side checks of the benchmark script (no GPU): the multi-GPU request is
refused with a message, the roofline helpers compute what they claim, and the
committed counter summaries are only used while they match the sources."""

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       stdout=subprocess.PIPE, stderr=subprocess.PIPE, timeout=120)
    assert r.returncode == 2
    assert b"one GPU" in r.stderr
    assert r.stdout == b""


def test_bandwidth_helper():
    # 36 B x 2^26 in 0.3019898 ms is 8 TB/s
    ms = 36 * bench.N_STREAM / 8000.0 / 1e6
    bw = bench._bandwidth(36, ms)
    assert bw["gbytes_per_s"] == pytest.approx(8000.0, rel=1e-6)
    assert bw["frac_of_hbm_peak"] == pytest.approx(1.0, abs=1e-4)


def test_committed_counter_summaries_are_tied_to_the_sources(tmp_path, monkeypatch):
    # the traffic figure is reported only while the recorded digest matches
    rec = json.load(open(os.path.join(ROOT, "profiles", "stream_sampler_2p26_counters.json")))
    t = bench.measured_traffic()
    if rec["source_digest"] == bench.source_digest():
        assert t == rec["hbm_bytes_per_launch"]
        assert abs(t / rec["algorithmic_bytes_per_launch"] - 1) < 1e-3
    else:
        assert t is None
    # a stale digest turns the figure off
    monkeypatch.setattr(bench, "source_digest", lambda: "0" * 16)
    assert bench.measured_traffic() is None


def test_alu_roofline_arithmetic():
    r = bench.alu_roofline("value_and_grad", 4096 * 2 ** 20, 12.8)
    if r is None:
        pytest.skip("VALU counter summary not taken on the current sources")
    ips = r["lane_instr_per_sample"]
    assert r["achieved"] == pytest.approx(ips * 4096 * 2 ** 20 / 12.8e-3 / 1e12, rel=1e-3)
    assert r["peak"] == pytest.approx(256 * 128 * 2.4e9 / 1e12, rel=1e-4)
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"], rel=1e-3)
