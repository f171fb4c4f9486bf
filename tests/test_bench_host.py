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


def test_batch_roofline_proxy_is_labelled():
    """The batch line's proxy prices its samples at another kernel's count and
    says so, with the same figures as that kernel's roofline."""
    assert bench.batch_kernel((512, 64, 8, 0, 1)) == "batch:k_batch<512, true, true>"
    r = bench.proxy_roofline("value_and_grad", 2073825747, 6.5)
    ref = bench.alu_roofline("value_and_grad", 2073825747, 6.5)
    if ref is None:
        assert r is None
        pytest.skip("VALU counter summary not taken on the current sources")
    assert r["per_sample_count_of"] == "value_and_grad"
    assert {k: v for k, v in r.items() if k != "per_sample_count_of"} == ref


FIXTURE = os.path.join(ROOT, "tests", "fixtures", "rocprof")


def test_profile_summaries_from_rocprof_csv(tmp_path):
    """--summarize-profiles on a trimmed copy of real rocprofv3 CSV output:
    the trace average, the counter calibration and the lane-instructions per
    sample are the arithmetic the summaries claim."""
    import csv
    import numpy as np
    done = bench.summarize_profiles(FIXTURE, prof=str(tmp_path), batch_samples=2073825747)
    assert done == ["stream_sampler_2p26", "stream_sampler_2p26_counters", "albedo_valu_counters"]
    # trace: the headline kernel's mean duration
    rows = list(csv.DictReader(open(os.path.join(FIXTURE, "trace", "run_kernel_trace.csv"))))
    dur = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in rows
           if "k_sample_v4<2," in r["Kernel_Name"]]
    rec = json.load(open(tmp_path / "stream_sampler_2p26.json"))
    assert rec["kernel"] == "k_sample_v4<2, false, true, 1>"
    assert rec["trace_avg_us"] == pytest.approx(np.mean(dur) / 1e3, abs=0.01)
    assert rec["frac_trace"] == pytest.approx(36 * 2 ** 26 / (np.mean(dur) * 1e-9) / 8e12,
                                              abs=1e-4)
    plain = json.load(open(os.path.join(FIXTURE, "bench_plain.json")))
    assert rec["event_ms_same_box"] == plain["ms_per_step"]
    assert "$REPO/bench.py --only stream fp32 disk probe" in rec["command_trace"]
    # traffic: calibration by the probe whose traffic is known
    def mean_counter(sub, kernel, name):
        rs = list(csv.DictReader(open(os.path.join(FIXTURE, sub, "run_counter_collection.csv"))))
        return np.mean([float(r["Counter_Value"]) for r in rs
                        if kernel in r["Kernel_Name"] and r["Counter_Name"] == name])
    t = json.load(open(tmp_path / "stream_sampler_2p26_counters.json"))
    fs = 20 * 2 ** 26 / 1024 / mean_counter("fetch", "k_stream_probe<0>", "FETCH_SIZE")
    ws = 16 * 2 ** 26 / 1024 / mean_counter("write", "k_stream_probe<0>", "WRITE_SIZE")
    assert t["fetch_scale"] == pytest.approx(fs) and t["write_scale"] == pytest.approx(ws)
    head = (mean_counter("fetch", "k_sample_v4<2,", "FETCH_SIZE") * fs +
            mean_counter("write", "k_sample_v4<2,", "WRITE_SIZE") * ws) * 1024
    assert t["hbm_bytes_per_launch"] == pytest.approx(head)
    assert abs(head / (36 * 2 ** 26) - 1) < 1e-3
    # VALU: SQ_INSTS_VALU x 64 / samples of one dispatch
    v = json.load(open(tmp_path / "albedo_valu_counters.json"))
    ips = v["valu_lane_instr_per_sample"]
    assert ips["forward_two_sums"] == pytest.approx(
        mean_counter("valu_a", "k_albedo_fwd<0>", "SQ_INSTS_VALU") * 64 / (4096 * 2 ** 20))
    assert ips["batch:k_batch<256, true, true>"] == pytest.approx(
        mean_counter("valu_b", "k_batch<256, true, true>", "SQ_INSTS_VALU") * 64 / 2073825747)
    assert 60 < ips["forward_two_sums"] < 90 and 120 < ips["value_and_grad"] < 180
