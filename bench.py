"""Benchmark of the spherical-cap GGX VNDF hot path on one MI355X.

One step = one launch of the streaming cap sampler over 2^26 anisotropic
tuples (FP32 structure of arrays in HBM, Philox uniforms drawn in-kernel,
outputs h and its pdf), in the method whose every output is within 2e-6 of
the exact sample: the cap sample evaluated in double precision from the FP32
inputs (CAPVNDF_CAP_F64).  The JSON line's value is that sampler's throughput
in Gsamples/s; alongside it the line reports the same sampler in FP32
arithmetic, the Heitz-2018 disk sampler on the same inputs, per-launch
medians and percentiles over at least 100 launches, the register-resident
cap-vs-disk microbenchmark, the directional-albedo table forward+backward
time, the batched estimator against per-request launches, the roofline of the
streaming kernel (from events, and from the committed kernel trace of the
same command), and -- in the CPU leg, the only part that runs the FP64
oracle -- the oracle timed on the host's CPU share, with the estimators'
errors against the oracle's stored values for every cell and job.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--only SECTION ...]
           [--no-cpu-baseline]
       python bench.py --summarize-profiles DIR   (rocprofv3 CSVs -> profiles/)
"""

import argparse
import csv
import glob
import hashlib
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("Gsamples/s VNDF (cap vs 2018 disk) + albedo-LUT fwd+bwd time at "
          "≤1e-4 err")
N_STREAM = 1 << 26
BYTES_PER_SAMPLE = 36  # 5 FP32 inputs read + 4 FP32 outputs written
HBM_PEAK_GBS = 8000.0
HEADLINE_METHOD = 2    # CAPVNDF_CAP_F64
MIN_LAUNCHES = 100     # per-launch statistics of the streaming kernels
MIN_EST_STEPS = 10     # timed launches of the estimator sections
SETTLE_LAUNCHES = 500  # untimed launches of the headline kernel before its warm-up
SECTIONS = ("plain", "stream", "fp32", "disk", "probe", "inverse", "dielectric", "micro", "lut",
            "grad", "batch", "radiance")
GOLDEN = os.path.join(ROOT, "tests", "golden", "estimator_full.npz")


def _lobes4():
    import numpy as np
    # four spherical-Gaussian lobes (mu_x, mu_y, mu_z, kappa, lambda)
    return np.array([[0.0, 0.0, 1.0, 4.0, 2.0], [0.6, 0.0, 0.8, 30.0, 5.0],
                     [-0.5, 0.5, 0.70710678, 10.0, 1.5], [0.0, 0.0, 1.0, 0.0, 0.3]],
                    dtype=np.float32)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--only", nargs="*", default=None, choices=SECTIONS)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-short-jobs", action="store_true",
                    help="batch section: leave out the short-job mix")
    ap.add_argument("--no-plain-pipeline", action="store_true",
                    help="batch section: leave out the per-request plain-sampler pipeline "
                         "(about 28k launches per pass and a graph of as many nodes; the "
                         "counter passes, which only need the batch kernels, skip it)")
    ap.add_argument("--summarize-profiles", metavar="DIR", default=None)
    ap.add_argument("--oracle-full-table", action="store_true",
                    help="CPU leg: run the oracle over the whole 64 x 64 x 2^20 table, timed, "
                         "and compare every cell live (about a minute on 16 threads)")
    return ap.parse_args(argv)


def _bandwidth(bytes_per_element, ms):
    """GB/s of a streaming launch over the 2^26-element workload, and its
    fraction of the 8 TB/s HBM peak."""
    gbs = bytes_per_element * N_STREAM / ms / 1e6
    return {"gbytes_per_s": round(gbs, 1), "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}


def timed(fn, steps, warmup):
    """Mean ms per call of fn over exactly `steps` calls on the current
    stream, with events recorded on that stream and device synchronisation on
    both sides; also the host's wall time per call."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    return e0.elapsed_time(e1) / steps, wall


def launch_stats(fn, launches):
    """Per-launch ms of `launches` back-to-back calls (an event pair on the
    launching stream around each): median, 10th and 90th percentile, mean."""
    import numpy as np
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(launches)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    ms = np.array([a.elapsed_time(b) for a, b in ev])
    return {"launches": launches, "median_ms": round(float(np.median(ms)), 5),
            "p10_ms": round(float(np.percentile(ms, 10)), 5),
            "p90_ms": round(float(np.percentile(ms, 90)), 5),
            "mean_ms": round(float(ms.mean()), 5)}


def source_digest():
    h = hashlib.sha256()
    for f in ("sample.hip", "device_math.hpp", "stream_io.hpp"):
        with open(os.path.join(ROOT, "paper_2306_05044_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the streaming kernel from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "stream_sampler_2p26_counters.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_digest") != source_digest():
        return None
    return rec.get("hbm_bytes_per_launch")


def alu_roofline(kind, samples, ms):
    """VALU roofline of an estimator kernel: lane-instructions per sample from
    the committed counter summary (if taken on the current sources) times the
    samples of one launch, over its launch time, against 256 CUs x 128 FP32
    lanes/clock x 2.4 GHz."""
    path = os.path.join(ROOT, "profiles", "albedo_valu_counters.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    h = hashlib.sha256()
    for name in ("albedo.hip", "albedo_math.hpp", "device_math.hpp"):
        with open(os.path.join(ROOT, "paper_2306_05044_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    if rec.get("source_digest") != h.hexdigest()[:16]:
        return None
    ips = rec["valu_lane_instr_per_sample"].get(kind)
    if ips is None:
        return None
    peak = rec["peak_lane_instr_per_s"] / 1e12
    achieved = ips * samples / (ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": round(achieved, 2), "peak": round(peak, 2),
            "unit": "T VALU lane-instr/s", "frac": round(achieved / peak, 4),
            "lane_instr_per_sample": round(ips, 1)}


def proxy_roofline(kind, samples, ms):
    """alu_roofline of a kernel priced at another kernel's per-sample count,
    labelled with that kernel's key; None where alu_roofline is None."""
    r = alu_roofline(kind, samples, ms)
    return None if r is None else {"per_sample_count_of": kind, **r}


def batch_kernel(tiling):
    """Counter-summary key of the batch kernel a tiling (block, pairs per
    thread, blocks per CU, per_wave, dynamic) runs, with gradients."""
    block, _, _, per_wave, dynamic = tiling
    name = "k_batch_wave" if per_wave else "k_batch"
    return f"batch:{name}<{block}, true, {'true' if dynamic else 'false'}>"


def trace_figures():
    """Kernel-trace figures of the headline kernel from the committed summary
    of a traced run of this benchmark (taken with a plain run of the same
    command on the same box), if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "stream_sampler_2p26.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_digest") != source_digest():
        return None
    return {k: rec[k] for k in ("kernel", "trace_avg_us", "trace_median_us", "frac_trace",
                                "trace_timed_region_avg_us", "frac_trace_timed_region",
                                "event_ms_same_box", "frac_event_same_box") if k in rec} | {
        "source": "profiles/stream_sampler_2p26.md"}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_share():
    """Host threads the oracle may use: the CPUs this process may run on,
    limited by a cgroup CPU quota if one is set, and by the 16 CPUs a GPU machine
    allots to one GPU; plus what the host reports."""
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    quota = None
    try:
        with open("/sys/fs/cgroup/cpu.max") as f:
            q, per = f.read().split()[:2]
            if q != "max":
                quota = int(q) / int(per)
    except (OSError, ValueError):
        pass
    share = aff if quota is None else max(1, min(aff, int(math.floor(quota))))
    threads = min(share, 16)
    return threads, {"os_cpu_count": os.cpu_count(), "affinity_cpus": aff,
                     "cgroup_cpu_quota": quota, "cpu_model": cpu_model()}


def cpu_baseline(d):
    """FP64 oracle on the host's CPU share: the full 2^26-tuple workload of
    the streaming configuration (cap sampler + pdf, Philox uniforms)."""
    import numpy as np
    import oracle
    threads, host = cpu_share()
    n = N_STREAM
    wi = tuple(d[k].astype(np.float64) for k in ("wx", "wy", "wz"))
    ax = d["ax"].astype(np.float64)
    ay = d["ay"].astype(np.float64)
    runs = []
    for _ in range(3):
        t0 = time.perf_counter()
        oracle.vndf_sample(wi, ax, ay, seed=1, method=0, nthreads=threads)
        runs.append(time.perf_counter() - t0)
    dt = sorted(runs)[1]
    return {"value": round(n / dt / 1e9, 6), "unit": "Gsamples/s", "cores": threads,
            "kind": "oracle", **host,
            "sample": f"all {n} tuples of the streaming workload, FP64 cap sampler + pdf; "
                      f"median of 3 runs ({dt:.2f} s each on {threads} host threads)"}


def load_golden():
    """The oracle's stored values for every cell and job of the estimator
    workloads (tests/golden/make_estimator_golden.py), keyed by workload, each
    only if the digest of its inputs matches the inputs generated now."""
    import importlib.util
    import numpy as np
    try:
        spec = importlib.util.spec_from_file_location(
            "make_estimator_golden", os.path.join(ROOT, "tests", "golden",
                                                  "make_estimator_golden.py"))
        mk = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mk)
        with np.load(GOLDEN, allow_pickle=False) as f:
            data = {k: f[k] for k in f.files}
    except (OSError, ValueError, ImportError):
        return {}
    out = {}
    for part, gen in (("lut", mk.lut_inputs), ("grad", mk.grad_inputs),
                      ("batch", mk.batch_inputs), ("radiance", mk.radiance_inputs)):
        if f"{part}_digest" in data and str(data[f"{part}_digest"]) == mk.digest(gen()):
            out[part] = data
    return out


def _grad_ratio(got, ref):
    import numpy as np
    return max(float((np.abs(g_ - r_) / (1e-4 + 1e-3 * np.abs(r_))).max())
               for g_, r_ in zip(got, ref))


def oracle_checks(checks):
    """The CPU leg's second part.  Every cell and job the estimator sections
    computed against the oracle's stored values for them (computed once with
    the oracle on the same inputs and Philox streams), and the oracle run live
    at a few cells, timed."""
    import numpy as np
    import oracle
    errs = {}
    gold = load_golden()
    threads, _ = cpu_share()
    if "plain_65536" in checks:
        c = checks["plain_65536"]
        d0 = c["inputs"]
        wi = tuple(d0[k].astype(np.float64) for k in ("wx", "wy", "wz"))
        t0 = time.perf_counter()
        h_ref, p_ref = oracle.vndf_sample(wi, d0["ax"], d0["ay"], seed=0, nthreads=threads)
        dt = time.perf_counter() - t0
        h = np.stack(c["got"][:3], axis=1).astype(np.float64)
        herr = float(np.linalg.norm(h - h_ref, axis=1).max())
        perr = float(np.abs(c["got"][3].astype(np.float64) / p_ref - 1.0).max())
        errs["plain_65536"] = {"oracle_seconds": round(dt, 3), "oracle_threads": threads,
                               "max_abs_err_h": herr, "max_rel_err_pdf": perr,
                               "every_tuple_within_2e-6": herr <= 2e-6 and perr <= 2e-6}
    if "albedo_lut" in checks:
        c = checks["albedo_lut"]
        r = {}
        if "lut" in gold:
            G = gold["lut"]
            r["every_cell"] = {
                "cells": 4096,
                "max_abs_err_s1": float(f"{np.abs(c['s1'] - G['lut_s1']).max():.3e}"),
                "max_abs_err_s5": float(f"{np.abs(c['s5'] - G['lut_s5']).max():.3e}"),
                "max_abs_err_a004": float(f"{np.abs(c['a004'] - G['lut_value']).max():.3e}"),
                "max_grad_err_over_tolerance": round(_grad_ratio(
                    c["g004"], (G["lut_gax"], G["lut_gay"], G["lut_gth"])), 4),
                "oracle_full_table_s1": {
                    "seconds": round(float(G["lut_s1_seconds"]), 1),
                    "threads": int(G["host_threads"]), "cpu_model": str(G["host_cpu_model"]),
                    "gsamples_per_s": round(4096 * (1 << 20) / float(G["lut_s1_seconds"]) / 1e9,
                                            4)}}
        if c.get("full_table"):
            g = c["grid"]
            t0 = time.perf_counter()
            f1 = oracle.albedo((g["wx"], g["wy"], g["wz"]), g["ax"], g["ay"], c["n"], 2,
                               f0=1.0, nthreads=threads)
            dt = time.perf_counter() - t0
            r["oracle_full_table_live"] = {
                "seconds": round(dt, 2), "threads": threads, "cpu_model": cpu_model(),
                "gsamples_per_s": round(4096 * c["n"] / dt / 1e9, 4),
                "max_abs_err_s1_every_cell": float(f"{np.abs(c['s1'] - f1).max():.3e}")}
        cells = np.linspace(0, 4095, 16).astype(np.int64)
        g = {k: v[cells] for k, v in c["grid"].items()}
        t0 = time.perf_counter()
        a1 = oracle.albedo((g["wx"], g["wy"], g["wz"]), g["ax"], g["ay"], c["n"], 2, f0=1.0,
                           units=cells, nthreads=threads)
        dt = time.perf_counter() - t0
        ns = len(cells) * c["n"]
        r["max_abs_err_vs_live_oracle"] = float(f"{np.abs(c['s1'][cells] - a1).max():.3e}")
        r["oracle"] = {"gsamples_per_s": round(ns / dt / 1e9, 6),
                       "cores": min(threads, len(cells)), "kind": "oracle",
                       "sample": f"{len(cells)} cells x {c['n']} samples, FP64 estimator, "
                                 f"one Fresnel sum ({dt:.2f} s)"}
        errs["albedo_lut"] = r
    if "albedo_grad" in checks and "grad" in gold:
        c = checks["albedo_grad"]
        G = gold["grad"]
        errs["albedo_grad"] = {"every_cell": {
            "cells": 1024, "path": "albedo_value_and_grad on the oracle's inputs",
            "max_abs_err": float(f"{np.abs(c['got'][0] - G['grad_value']).max():.3e}"),
            "max_grad_err_over_tolerance": round(_grad_ratio(
                c["got"][1:], (G["grad_gax"], G["grad_gay"], G["grad_gth"])), 4)}}
    if "batched" in checks:
        c = checks["batched"]
        r = {}
        if "batch" in gold:
            G = gold["batch"]
            for mode in ("graph", "per_request"):
                got = c[mode]
                r[f"every_job_{mode}"] = {
                    "jobs": 4096,
                    "max_abs_err": float(f"{np.abs(got[0] - G['batch_value']).max():.3e}"),
                    "max_grad_err_over_tolerance": round(_grad_ratio(
                        got[1:], (G["batch_gax"], G["batch_gay"], G["batch_gth"])), 4)}
            r["oracle_every_job"] = {"seconds": round(float(G["batch_seconds"]), 1),
                                     "threads": int(G["host_threads"]),
                                     "cpu_model": str(G["host_cpu_model"]),
                                     "what": "FP64 value + dual-number gradient, all jobs"}
        errs["batched"] = r
    if "direct_illumination" in checks:
        c = checks["direct_illumination"]
        g = c["grid"]
        ref = oracle.radiance((g["wx"], g["wy"], g["wz"]), g["ax"], g["ay"], c["n"], 2,
                              c["lobes"].astype(np.float64), units=c["cells"])
        errs["direct_illumination"] = {
            "max_abs_err_vs_oracle": float(f"{np.abs(c['value'] - ref).max():.3e}"),
            "err_checked_cells": len(c["cells"])}
        if "radiance" in gold and np.array_equal(gold["radiance"]["radiance_lobes"],
                                                 c["lobes"]):
            G = gold["radiance"]
            errs["direct_illumination"]["every_cell"] = {
                "cells": 4096,
                "max_abs_err": float(f"{np.abs(c['all'] - G['radiance_value']).max():.3e}"),
                "tolerance": float(f"{1e-4 * float(c['lobes'][:, 4].sum()):.3e}"),
                "oracle_seconds": round(float(G["radiance_seconds"]), 1),
                "oracle_threads": int(G["host_threads"])}
    return errs


def _stream_entry(ms, stats, bytes_per_sample=BYTES_PER_SAMPLE):
    return {"ms_per_launch": round(ms, 5), "gsamples_per_s": round(N_STREAM / ms / 1e6, 3),
            **_bandwidth(bytes_per_sample, ms), "launch_stats": stats}


# ---------------------------------------------------------------------------
# --summarize-profiles DIR: turn the rocprofv3 CSV output of the profiling
# passes (each taken on the benchmark itself) into the summaries under
# profiles/ that the JSON line reads (traffic, trace and VALU figures).
#
# DIR holds one folder per pass, each the `-d` of one rocprofv3 run with
# `--output-format csv`:
#   trace/   --kernel-trace --stats  of  bench.py --only stream fp32 disk probe
#   fetch/   --pmc FETCH_SIZE        of  the same sections (fewer steps)
#   write/   --pmc WRITE_SIZE        of  the same sections (fewer steps)
#   valu_a/  --pmc <VALU counters>   of  bench.py --only micro lut radiance
#   valu_b/  (optional) --pmc <VALU counters> --kernel-include-regex
#            (k_batch|k_radiance|k_horizon_fix) of bench.py --only batch ...
# and bench_plain.json (the JSON line of the traced command run without the
# profiler, same box) and commands.txt ("<pass>: <command>" per line).
# ---------------------------------------------------------------------------
STREAM_KERNELS = {  # kernel-name prefix -> (label, algorithmic bytes per element)
    "k_sample_v4<2,": ("cap sampler, double-precision arithmetic (headline)", 36),
    "k_sample_v4<0,": ("cap sampler, FP32 arithmetic", 36),
    "k_sample_v4<1,": ("Heitz-2018 disk sampler, FP32", 36),
    "k_stream_probe<0>": ("streaming probe: the sampler's traffic", 36),
    "k_stream_probe<1>": ("streaming probe: reads only", 20),
    "k_stream_probe<2>": ("streaming probe: writes only", 16),
}
VALU_COUNTERS = ("SQ_INSTS_VALU", "SQ_INSTS_VALU_TRANS_F32", "SQ_INSTS_VALU_INT64",
                 "SQ_INSTS_SALU", "SQ_BUSY_CYCLES", "SQ_WAVES", "GRBM_GUI_ACTIVE")
VALU_PEAK = 256 * 128 * 2.4e9  # FP32 lanes x clock: the issue rate behind 157.3 TFLOP/s
ESTIMATOR_MICRO_LANES, ESTIMATOR_MICRO_PAIRS = 256 * 2048 * 4, 32
ESTIMATOR_MICRO_SAMPLES = ESTIMATOR_MICRO_LANES * 2 * ESTIMATOR_MICRO_PAIRS


def _short_name(name):
    """Kernel name without namespaces, return type and parameter list."""
    n = name.replace("capvndf::(anonymous namespace)::", "").replace("capvndf::", "").strip()
    if n.startswith("void "):
        n = n[5:]
    depth = 0
    for i, ch in enumerate(n):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return n[:i].strip()
    return n


def _csv(folder, suffix):
    hits = sorted(glob.glob(os.path.join(folder, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {folder}")
    with open(hits[0], newline="") as f:
        return list(csv.DictReader(f))


def _col(row, *names):
    for n in names:
        if n in row:
            return row[n]
    raise KeyError(f"none of {names} in {sorted(row)}")


def trace_rows(folder):
    """{short kernel name: [(start ns, duration ns, grid work-items), ...]}
    from a kernel-trace CSV, each list in start order."""
    out = {}
    for r in _csv(folder, "kernel_trace.csv"):
        k = _short_name(_col(r, "Kernel_Name", "Name"))
        start = int(_col(r, "Start_Timestamp"))
        dur = int(_col(r, "End_Timestamp")) - start
        out.setdefault(k, []).append((start, dur, int(float(_col(r, "Grid_Size_X", "Grid_Size")))))
    return {k: sorted(v) for k, v in out.items()}


def read_trace(folder):
    """{short kernel name: [duration ns, ...]} from a kernel-trace CSV, in
    start order."""
    return {k: [d for _, d, _ in v] for k, v in trace_rows(folder).items()}


def read_counters(folder):
    """{short kernel name: [{counter: value, "grid": work-items}, ...]} per
    dispatch from a counter-collection CSV."""
    per = {}
    for r in _csv(folder, "counter_collection.csv"):
        key = (_col(r, "Dispatch_Id", "Correlation_Id"), _short_name(_col(r, "Kernel_Name")))
        d = per.setdefault(key, {"grid": int(float(_col(r, "Grid_Size", "Grid_Size_X")))})
        d[_col(r, "Counter_Name")] = d.get(_col(r, "Counter_Name"), 0.0) + \
            float(_col(r, "Counter_Value"))
    out = {}
    for (_, k), d in sorted(per.items(), key=lambda kv: int(kv[0][0])):
        out.setdefault(k, []).append(d)
    return out


def _commands(d):
    cmds = {}
    path = os.path.join(d, "commands.txt")
    if os.path.exists(path):
        for line in open(path):
            if ":" in line:
                k, v = line.split(":", 1)
                cmds[k.strip()] = v.strip()
    return cmds


def _kernel(rows, prefix):
    for k in rows:
        if k.startswith(prefix):
            return k
    return None


def _valu_digest():
    h = hashlib.sha256()
    for name in ("albedo.hip", "albedo_math.hpp", "device_math.hpp"):
        with open(os.path.join(ROOT, "paper_2306_05044_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def summarize_stream(d, cmds, prof):
    import numpy as np
    rows = trace_rows(os.path.join(d, "trace"))
    with open(os.path.join(d, "bench_plain.json")) as f:
        plain = json.loads(f.read().strip().splitlines()[-1])
    head = _kernel(rows, "k_sample_v4<2,")
    # the 2^26-tuple launches only (the largest grid of the kernel)
    big = max(g for _, _, g in rows[head])
    tr = {k: [dd for _, dd, gg in v if gg == max(g for _, _, g in v)] for k, v in rows.items()}
    dur = np.array(tr[head], dtype=np.float64) / 1e3
    algo = BYTES_PER_SAMPLE * N_STREAM
    # The headline's launches in a traced run: the settling launches, the
    # warm-up, the timed region (`steps` back-to-back launches, the line's
    # ms_per_step), then the separately bracketed ones of launch_stats.
    region = None
    if all(k in plain for k in ("steps", "warmup")):
        skip = int(plain.get("settle_launches", 0)) + int(plain["warmup"])
        if dur.size >= skip + int(plain["steps"]):
            region = dur[skip:skip + int(plain["steps"])]
    rec = {"source_digest": source_digest(), "kernel": head,
           "trace_dispatches": int(dur.size), "trace_avg_us": round(float(dur.mean()), 2),
           "trace_median_us": round(float(np.median(dur)), 2),
           "trace_min_us": round(float(dur.min()), 2), "trace_max_us": round(float(dur.max()), 2),
           "frac_trace": round(algo / (dur.mean() * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
           "grid_work_items": big,
           "trace_timed_region_avg_us": None if region is None else round(float(region.mean()), 2),
           "frac_trace_timed_region": None if region is None else
           round(algo / (region.mean() * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
           "event_ms_same_box": plain["ms_per_step"],
           "frac_event_same_box": plain["roofline"]["frac"],
           "event_median_ms_same_box": plain["launch_stats"]["median_ms"],
           "command_trace": cmds.get("trace", ""), "command_plain": cmds.get("plain", "")}
    with open(os.path.join(prof, "stream_sampler_2p26.json"), "w") as f:
        json.dump(rec, f, indent=1)
    lines = ["# Kernel trace of the streaming samplers (2^26 tuples)", "",
             "MI355X (gfx950).  The benchmark's streaming sections, traced, and the same command "
             "without the profiler on the same box:", "", "```",
             cmds.get("trace", "(command not recorded)"), cmds.get("plain", ""), "```", "",
             "| kernel | what | dispatches | avg (us) | median (us) | min (us) | max (us) | "
             "GB/s at avg | of 8 TB/s |", "|---|---|---|---|---|---|---|---|---|"]
    for pre, (label, bpe) in STREAM_KERNELS.items():
        k = _kernel(tr, pre)
        if k is None:
            continue
        x = np.array(tr[k], dtype=np.float64) / 1e3
        gbs = bpe * N_STREAM / (x.mean() * 1e-6) / 1e9
        lines.append(f"| `{k}` | {label} | {x.size} | {x.mean():.2f} | {np.median(x):.2f} | "
                     f"{x.min():.2f} | {x.max():.2f} | {gbs:.0f} | {gbs / HBM_PEAK_GBS:.1%} |")
    lines += ["", f"Headline kernel `{head}`: trace average {rec['trace_avg_us']:.2f} us over all "
              f"its {rec['trace_dispatches']} launches, including the settling ones "
              f"(fraction of the HBM peak {rec['frac_trace']:.4f})"
              + ("" if region is None else
                 f"; over the {region.size} launches of the timed region "
                 f"{rec['trace_timed_region_avg_us']:.2f} us (fraction "
                 f"{rec['frac_trace_timed_region']:.4f})") + "; the benchmark's own event "
              f"timing on the same box: {rec['event_ms_same_box'] * 1e3:.2f} us per launch over "
              f"the timed region (fraction {rec['frac_event_same_box']:.4f}), per-launch median "
              f"{rec['event_median_ms_same_box'] * 1e3:.2f} us.",
              f"`bench.py` reports these trace figures while the digest of `csrc/sample.hip` + "
              f"`csrc/device_math.hpp` + `csrc/stream_io.hpp` equals `{rec['source_digest']}`.",
              "", f"Written by `python bench.py --summarize-profiles <dir>`."]
    with open(os.path.join(prof, "stream_sampler_2p26.md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    return rec


def summarize_traffic(d, cmds, prof):
    import numpy as np
    fe = read_counters(os.path.join(d, "fetch"))
    wr = read_counters(os.path.join(d, "write"))

    def mean(rows, k, c):
        return float(np.mean([r[c] for r in rows[k]]))
    probe = _kernel(fe, "k_stream_probe<0>")
    known_fetch, known_write = 20 * N_STREAM / 1024, 16 * N_STREAM / 1024  # KiB
    fs = known_fetch / mean(fe, probe, "FETCH_SIZE")
    ws = known_write / mean(wr, probe, "WRITE_SIZE")
    rec = {"source_digest": source_digest(), "fetch_scale": fs, "write_scale": ws,
           "algorithmic_bytes_per_launch": BYTES_PER_SAMPLE * N_STREAM, "kernels": {}}
    lines = ["# HBM traffic of the streaming kernels (2^26 elements), rocprofv3 counters", "",
             "Two counter passes (one counter each), MI355X (gfx950):", "", "```",
             cmds.get("fetch", ""), cmds.get("write", ""), "```", "",
             "Counters are KiB per dispatch (mean over the dispatches of each kernel).  "
             "Calibration with `k_stream_probe<0>`, whose traffic is known exactly (20 B read "
             "and 16 B written per element): "
             f"FETCH_SIZE scale = {fs:.6f}, WRITE_SIZE scale = {ws:.6f}.", "",
             "| kernel | algorithmic B / element | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) | "
             "HBM bytes / launch, scaled (GB) | / algorithmic |", "|---|---|---|---|---|---|"]
    for pre, (label, bpe) in STREAM_KERNELS.items():
        k = _kernel(fe, pre)
        if k is None or _kernel(wr, pre) is None:
            continue
        f_, w_ = mean(fe, k, "FETCH_SIZE"), mean(wr, _kernel(wr, pre), "WRITE_SIZE")
        hbm = (f_ * fs + w_ * ws) * 1024
        rec["kernels"][k] = {"hbm_bytes_per_launch": hbm, "bytes_per_element": bpe,
                             "fetch_kib": f_, "write_kib": w_}
        lines.append(f"| `{k}` | {bpe} | {f_:,.1f} | {w_:,.1f} | {hbm / 1e9:.4f} | "
                     f"{hbm / (bpe * N_STREAM):.4f} |")
    head = _kernel(fe, "k_sample_v4<2,")
    rec["hbm_bytes_per_launch"] = rec["kernels"][head]["hbm_bytes_per_launch"]
    with open(os.path.join(prof, "stream_sampler_2p26_counters.json"), "w") as f:
        json.dump(rec, f, indent=1)
    lines += ["", f"`bench.py` reports `roofline.traffic` (the headline kernel's row) while the "
              f"source digest equals `{rec['source_digest']}`.", "",
              "Written by `python bench.py --summarize-profiles <dir>`."]
    with open(os.path.join(prof, "stream_sampler_2p26_counters.md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    return rec


def summarize_valu(d, cmds, prof, batch_samples):
    """Lane-instructions per sample of the estimators and the microbenchmark
    from SQ counters; samples per dispatch from the workloads' sizes."""
    import numpy as np
    a = read_counters(os.path.join(d, "valu_a"))
    # the batch kernels' pass is optional (its own run, with the include regex)
    b = read_counters(os.path.join(d, "valu_b")) if os.path.isdir(os.path.join(d, "valu_b")) \
        else {}
    lut = 4096 * (1 << 20)
    # the 64x64 table's launches: 4096 cells x slots blocks of 256 work-items
    # (32 slots per cell; 64 in traces of builds before that change)
    lut_grids = {4096 * slots * 256 for slots in (32, 64)}
    micro = 256 * 2048 * 4 * 64
    rows = []  # (key, kernel, description, samples, [dispatch dicts])
    for pre, key, desc in (("k_albedo_fwd<0>", "forward_two_sums", "forward, two Fresnel sums"),
                           ("k_albedo_adj<false>", "backward", "backward (recompute)"),
                           ("k_albedo_adj<true>", "value_and_grad", "value + Jacobian, one pass")):
        k = _kernel(a, pre)
        if k:
            rows.append((key, k, desc + " (64x64 cells x 2^20)", lut,
                         [x for x in a[k] if x["grid"] in lut_grids]))
    # the horizon fix passes after the table's adjoint kernels: a wavefront
    # per 4 of a cell's 32 slots (per 8 of 64 in earlier builds), 4096 x 8
    # blocks of 64 work-items
    fix_grids = {4096 * 8 * 64}
    for pre, key, desc in (("k_horizon_fix_table<false>", "fix_backward",
                            "horizon fix after backward"),
                           ("k_horizon_fix_table<true>", "fix_value_and_grad",
                            "horizon fix after value + Jacobian")):
        k = _kernel(a, pre)
        if k:
            rows.append((key, k, desc + " (per table sample)", lut,
                         [x for x in a[k] if x["grid"] in fix_grids]))
    for m, name in ((0, "cap"), (1, "disk"), (2, "cap in double precision")):
        k = _kernel(a, f"k_microbench<{m}>")
        if k:
            rows.append((f"micro_{m}", k, f"microbenchmark, {name} (2^21 lanes x 64)", micro,
                         a[k]))
    for m, key, name in ((0, "mix_forward", "forward's two sums"),
                         (1, "mix_value_and_adjoint", "value and adjoint"),
                         (2, "mix_radiance", "radiance, 4 lobes")):
        k = _kernel(a, f"k_estimator_microbench<{m}>")
        if k:
            rows.append((key, k, f"register-resident estimator code: {name} (2^21 lanes x 64)",
                         ESTIMATOR_MICRO_SAMPLES, a[k]))
    src = b if _kernel(b, "k_radiance<4>") else a
    k = _kernel(src, "k_radiance<4>")
    if k:
        rows.append(("radiance", k, "direct illumination, 4 lobes (64x64 cells x 2^20)", lut,
                     [x for x in src[k] if x["grid"] in lut_grids]))
    for k in sorted(b):
        if k.startswith("k_batch"):
            rows.append((f"batch:{k}", k, "batch forward + adjoint, 4096 jobs", batch_samples,
                         b[k]))
        elif k.startswith("k_horizon_fix_batch"):
            rows.append((f"batch:{k}", k, "batch horizon fix (per batch sample)", batch_samples,
                         b[k]))
    rec = {"source_digest": _valu_digest(), "valu_lane_instr_per_sample": {},
           "peak_lane_instr_per_s": VALU_PEAK, "source": "profiles/albedo_valu_counters.md"}
    lines = ["# VALU counters of the estimators and the sampler microbenchmark", "",
             "MI355X (gfx950).  Commands (counter passes of the benchmark itself):", "", "```",
             *[cmds[k] for k in ("valu_a", "valu_b") if k in cmds], "```", "",
             "Counts per dispatch (mean over the dispatches listed).  VALU lane-instructions = "
             "`SQ_INSTS_VALU` x 64.  `GRBM_GUI_ACTIVE` is summed over the 8 XCDs, so busy "
             "time = value / 8 / 2.4 GHz.  Peak for the fraction: 256 CUs x 128 FP32 lanes x "
             "2.4 GHz = 78.6e12 lane-instructions/s.", "",
             "| kernel (workload) | dispatches | samples / dispatch | VALU lane-instr / sample | "
             "transcendental / sample | 64-bit int / sample | busy time (ms) | "
             "T lane-instr/s | of 78.6 T |", "|---|---|---|---|---|---|---|---|---|"]
    rates = {}
    for key, k, desc, ns, disp in rows:
        if not disp:
            continue
        mv = {c: float(np.mean([x.get(c, 0.0) for x in disp])) for c in VALU_COUNTERS}
        ips = mv["SQ_INSTS_VALU"] * 64 / ns
        busy_s = mv["GRBM_GUI_ACTIVE"] / 8 / 2.4e9
        rate = mv["SQ_INSTS_VALU"] * 64 / busy_s if busy_s > 0 else float("nan")
        rec["valu_lane_instr_per_sample"][key] = ips
        rates[key] = rate
        lines.append(f"| `{k}` {desc} | {len(disp)} | {ns:.4g} | {ips:.1f} | "
                     f"{mv['SQ_INSTS_VALU_TRANS_F32'] * 64 / ns:.2f} | "
                     f"{mv['SQ_INSTS_VALU_INT64'] * 64 / ns:.2f} | {busy_s * 1e3:.3f} | "
                     f"{rate / 1e12:.1f} | {rate / VALU_PEAK:.1%} |")
    ceil = {}
    for key, mix in (("forward_two_sums", "mix_forward"), ("value_and_grad", "mix_value_and_adjoint"),
                     ("radiance", "mix_radiance")):
        if key in rates and mix in rates:
            ceil[key] = {"mix_ceiling_lane_instr_per_s": rates[mix],
                         "frac_of_mix_ceiling": rates[key] / rates[mix]}
    rec["mix_ceiling"] = ceil
    if ceil:
        lines += ["", "Against the issue rate of the same per-sample code run register-resident "
                  "(`estimator_microbench`: no loads in the loop, no compensated sums, no "
                  "cross-lane reductions, the kernel's own occupancy):", "",
                  "| kernel | its rate (T/s) | mix ceiling (T/s) | fraction |", "|---|---|---|---|"]
        for key, v in ceil.items():
            lines.append(f"| {key} | {rates[key] / 1e12:.1f} | "
                         f"{v['mix_ceiling_lane_instr_per_s'] / 1e12:.1f} | "
                         f"{v['frac_of_mix_ceiling']:.1%} |")
    with open(os.path.join(prof, "albedo_valu_counters.json"), "w") as f:
        json.dump(rec, f, indent=1)
    lines += ["", f"`bench.py` reads the per-sample counts while the digest of "
              f"`csrc/albedo.hip` + `csrc/albedo_math.hpp` + `csrc/device_math.hpp` equals "
              f"`{rec['source_digest']}`.", "",
              "Written by `python bench.py --summarize-profiles <dir>`."]
    with open(os.path.join(prof, "albedo_valu_counters.md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    return rec


def summarize_profiles(d, prof=None, batch_samples=None):
    """Every summary whose passes are present under d."""
    prof = prof or os.path.join(ROOT, "profiles")
    cmds = _commands(d)
    done = []
    if os.path.isdir(os.path.join(d, "trace")):
        summarize_stream(d, cmds, prof)
        done.append("stream_sampler_2p26")
    if os.path.isdir(os.path.join(d, "fetch")) and os.path.isdir(os.path.join(d, "write")):
        summarize_traffic(d, cmds, prof)
        done.append("stream_sampler_2p26_counters")
    if os.path.isdir(os.path.join(d, "valu_a")):
        if batch_samples is None:
            import workloads
            batch_samples = int(workloads.batch_jobs(4096, seed=4)["n"].sum())
        summarize_valu(d, cmds, prof, batch_samples)
        done.append("albedo_valu_counters")
    log("summarized: " + ", ".join(done))
    return done


def main():
    args = parse()
    if args.summarize_profiles:
        summarize_profiles(args.summarize_profiles)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the path shards by "
              "tuple/cell/job ranges with no exchange but a final reduction, which this library "
              "does not run across GPUs.", file=sys.stderr)
        sys.exit(2)
    only = set(args.only) if args.only else set(SECTIONS)

    import numpy as np
    import torch
    import paper_2306_05044_amd as cv
    import workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cv.load_library()
    out = {}
    checks = {}  # GPU values, compared with the oracle in the CPU leg
    est_steps = max(MIN_EST_STEPS, args.steps // 10)
    LOBES4 = _lobes4()
    mix_ceiling = {}  # Gsamples/s of the register-resident estimator code
    nstats = max(MIN_LAUNCHES, args.steps)

    log("generating the 2^26-tuple streaming workload")
    d = workloads.tuples_streaming(N_STREAM, seed=1)
    t = {k: torch.from_numpy(v).to(dev) for k, v in d.items()}
    outs = tuple(torch.empty_like(t["wx"]) for _ in range(4))

    def run(method):
        return lambda: cv.vndf_sample(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], seed=1,
                                      method=method, out=outs)

    # The comparison sections run first: the first few hundred milliseconds
    # of sustained load on an idle GPU show a clock transient (launches up
    # to 1.5x slower for some 40 ms), which the headline's timed region is
    # kept out of.
    ms_32 = ms_disk = None
    if "plain" in only:
        # the plain sampler on its 65,536 isotropic tuples (Philox seed 0):
        # launch-bound on the GPU; the CPU leg runs the oracle over every
        # tuple, timed, and compares each output
        log("timing the plain sampler, 65,536 tuples")
        d0 = workloads.tuples_small(65536, seed=0)
        t0_ = {k: torch.from_numpy(v).to(dev) for k, v in d0.items()}
        outs0 = tuple(torch.empty_like(t0_["wx"]) for _ in range(4))

        def run0():
            cv.vndf_sample(t0_["wx"], t0_["wy"], t0_["wz"], t0_["ax"], t0_["ay"], seed=0,
                           method=HEADLINE_METHOD, out=outs0)
        for _ in range(args.warmup):
            run0()
        st0 = launch_stats(run0, 100)
        run0()
        torch.cuda.synchronize()
        out["plain_65536"] = {"tuples": 65536, "method": "cap_f64", "launch_stats": st0,
                              "gsamples_per_s": round(65536 / st0["median_ms"] / 1e6, 2)}
        checks["plain_65536"] = {"inputs": d0, "got": [o.cpu().numpy() for o in outs0]}
        del t0_, outs0
    if "fp32" in only:
        log("timing the cap sampler in FP32 arithmetic")
        ms_32, _ = timed(run(0), args.steps, args.warmup)
        out["cap_fp32"] = {"what": "the same samples in FP32 arithmetic (per-sample error "
                                   "bound 2^-24 times the conditioning, not a flat 2e-6)",
                           **_stream_entry(ms_32, launch_stats(run(0), nstats))}
    if "disk" in only:
        log("timing the disk-2018 sampler")
        ms_disk, _ = timed(run(1), args.steps, args.warmup)
        out["disk2018"] = {"what": "Heitz 2018 cross-section sampler, FP32 arithmetic, same "
                                   "inputs and uniforms",
                           **_stream_entry(ms_disk, launch_stats(run(1), nstats))}
        if ms_32:
            out["disk2018"]["t_disk_over_t_cap_fp32"] = round(ms_disk / ms_32, 4)
    if "probe" in only:
        log("timing the streaming probe")
        ins = [t[k] for k in ("wx", "wy", "wz", "ax", "ay")]
        ms_p, _ = timed(lambda: cv.capvndf_stream_probe(ins, outs), args.steps, args.warmup)
        ms_r, _ = timed(lambda: cv.capvndf_stream_probe(ins, outs, mode=1), args.steps,
                        args.warmup)
        ms_w, _ = timed(lambda: cv.capvndf_stream_probe(ins, outs, mode=2), args.steps,
                        args.warmup)
        out["stream_probe"] = {"ms_per_launch": round(ms_p, 5),
                               **_bandwidth(BYTES_PER_SAMPLE, ms_p),
                               "read_only_gbytes_per_s": round(20 * N_STREAM / ms_r / 1e6, 1),
                               "write_only_gbytes_per_s": round(16 * N_STREAM / ms_w / 1e6, 1)}
    ms_head = wall_head = head_stats = None
    if "stream" in only:
        log(f"timing the headline sampler (cap, double-precision arithmetic): {args.steps} "
            f"launches, then {nstats} with per-launch events")
        # Under the double-precision kernel's load the clock settles for some
        # 40 ms (launches up to 1.2x slower, recovering over about a hundred
        # launches): that settling happens before the warm-up steps.
        settle = run(HEADLINE_METHOD)
        for _ in range(SETTLE_LAUNCHES):
            settle()
        torch.cuda.synchronize()
        ms_head, wall_head = timed(run(HEADLINE_METHOD), args.steps, args.warmup)
        head_stats = launch_stats(run(HEADLINE_METHOD), nstats)
        log(f"cap_f64: {ms_head:.4f} ms/launch")
        if ms_32:
            out["cap_fp32"]["t_fp32_over_t_f64"] = round(ms_32 / ms_head, 4)
        if ms_disk:
            out["disk2018"]["t_disk_over_t_cap"] = round(ms_disk / ms_head, 4)
    if "inverse" in only:
        log("timing the inverse map h -> (u1, u2)")
        run(HEADLINE_METHOD)()
        u1b = torch.empty_like(t["wx"])
        u2b = torch.empty_like(t["wx"])
        ms_i, _ = timed(lambda: cv.vndf_inverse(t["wx"], t["wy"], t["wz"], outs[0], outs[1],
                                                outs[2], t["ax"], t["ay"], out=(u1b, u2b)),
                        args.steps, args.warmup)
        out["inverse_map"] = {"ms_per_launch": round(ms_i, 5),
                              "gsamples_per_s": round(N_STREAM / ms_i / 1e6, 3),
                              **_bandwidth(40, ms_i),
                              "bytes_per_sample": 40}
        log("timing the VNDF pdf at the sampled normals")
        ms_p, _ = timed(lambda: cv.vndf_pdf(t["wx"], t["wy"], t["wz"], outs[0], outs[1], outs[2],
                                            t["ax"], t["ay"], out=u1b), args.steps, args.warmup)
        out["vndf_pdf"] = {"ms_per_launch": round(ms_p, 5),
                           "gsamples_per_s": round(N_STREAM / ms_p / 1e6, 3),
                           **_bandwidth(36, ms_p),
                           "bytes_per_sample": 36}
        del u1b, u2b
    if "dielectric" in only:
        log("timing the rough-dielectric sampler and its pdf (eta = 1.5)")
        douts = (outs[0], outs[1], outs[2], outs[3], torch.empty_like(t["wx"]))
        ms_ds, _ = timed(lambda: cv.dielectric_sample(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"],
                                                      1.5, seed=1, out=douts),
                         args.steps, args.warmup)
        ms_dp, _ = timed(lambda: cv.dielectric_pdf(t["wx"], t["wy"], t["wz"], douts[0], douts[1],
                                                   douts[2], t["ax"], t["ay"], 1.5, out=douts[4]),
                         args.steps, args.warmup)
        out["dielectric"] = {
            "eta": 1.5,
            "sample": {"ms_per_launch": round(ms_ds, 5),
                       "gsamples_per_s": round(N_STREAM / ms_ds / 1e6, 3),
                       **_bandwidth(40, ms_ds),
                       "bytes_per_sample": 40},
            "pdf": {"ms_per_launch": round(ms_dp, 5),
                    "gsamples_per_s": round(N_STREAM / ms_dp / 1e6, 3),
                    **_bandwidth(36, ms_dp),
                    "bytes_per_sample": 36}}
        del douts
    if "micro" in only:
        log("timing the register-resident microbenchmark")
        lanes = 256 * 2048 * 4
        iters = 64
        buf = torch.empty(lanes, dtype=torch.int32, device=dev)
        res = {}
        methods = (("cap", 0), ("disk2018", 1), ("cap_f64", 2))
        # the methods alternate over several rounds of MIN_LAUNCHES launches
        # each, so that a drift of the clock during the run moves all of them
        # alike; medians over the rounds and per-launch percentiles reported
        rounds = {name: [] for name, _ in methods}
        stats = {name: [] for name, _ in methods}
        for _, m in methods:  # untimed: the first launches after a pause run on a cold clock
            timed(lambda: cv.vndf_microbench(m, lanes, iters, 1, out=buf), 50, 3)
        for _ in range(5):
            for name, m in methods:
                st = launch_stats(lambda: cv.vndf_microbench(m, lanes, iters, 1, out=buf),
                                  MIN_LAUNCHES)
                rounds[name].append(st["median_ms"])
                stats[name].append(st)
        for name, _ in methods:
            ms = float(np.median(rounds[name]))
            res[name] = {"median_ms": round(ms, 5),
                         "gsamples_per_s": round(lanes * iters / ms / 1e6, 2),
                         "p10_ms": round(float(np.median([x["p10_ms"] for x in stats[name]])), 5),
                         "p90_ms": round(float(np.median([x["p90_ms"] for x in stats[name]])), 5)}
        ratio = [dk / c for dk, c in zip(rounds["disk2018"], rounds["cap"])]
        res["t_disk_over_t_cap"] = round(float(np.median(ratio)), 4)
        res["t_disk_over_t_cap_rounds"] = [round(min(ratio), 4), round(max(ratio), 4)]
        # the double-precision cap's arithmetic without memory traffic to hide it
        res["t_cap_f64_over_t_cap"] = round(
            float(np.median([f / c for f, c in zip(rounds["cap_f64"], rounds["cap"])])), 4)
        res["lanes"] = lanes
        res["calls_per_lane"] = iters
        # the estimators' per-sample arithmetic, register-resident: the
        # ceiling of their instruction mix (the table sections divide by it)
        lobes4 = torch.from_numpy(LOBES4).to(dev)
        elanes, epairs = ESTIMATOR_MICRO_LANES, ESTIMATOR_MICRO_PAIRS
        est = {}
        for kind, name in ((0, "forward_two_sums"), (1, "value_and_adjoint"),
                           (2, "radiance_4_lobes")):
            st = launch_stats(lambda: cv.estimator_microbench(kind, elanes, epairs, 1, lobes4,
                                                              out=buf), MIN_LAUNCHES)
            est[name] = {"median_ms": st["median_ms"], "p10_ms": st["p10_ms"],
                         "p90_ms": st["p90_ms"],
                         "gsamples_per_s": round(elanes * 2 * epairs / st["median_ms"] / 1e6, 2)}
        est["what"] = (f"{elanes} lanes x {2 * epairs} samples of the estimator's per-sample "
                       "code into plain per-lane sums (no loads, no reductions)")
        res["estimator_mix"] = est
        mix_ceiling.update({k: v["gsamples_per_s"] for k, v in est.items() if k != "what"})
        res["rounds"] = f"5 alternating rounds of {MIN_LAUNCHES} launches per method"
        res["paper_speedups"] = {"Intel Arc A770": "52.96%", "NVIDIA RTX 2080": "39.25%",
                                 "Intel i7-13700K (CPU)": "37.67%"}
        out["microbench"] = res
    del t, outs
    torch.cuda.empty_cache()

    if "lut" in only:
        log("albedo table 64 x 64 x 2^20: forward, backward, one-pass value + gradient")
        g = workloads.lut_grid(64, 64)
        c = {k: torch.from_numpy(v).to(dev) for k, v in g.items()}
        n = 1 << 20
        counts = torch.full((4096,), n, dtype=torch.int64, device=dev)
        ws = torch.empty(cv.albedo_workspace_size(4096, np.full(4096, n), 1) // 4 + 4,
                         device=dev)
        f0 = torch.full((4096,), 0.04, device=dev)

        def fwd():
            return cv.albedo_estimate(c["wx"], c["wy"], c["wz"], c["ax"], c["ay"], counts, 2,
                                      workspace=ws)

        def bwd():
            return cv.albedo_estimate_backward(c["wx"], c["wy"], c["wz"], c["ax"], c["ay"],
                                               counts, 2, workspace=ws)

        def fused():
            return cv.albedo_value_and_grad(c["wx"], c["wy"], c["wz"], c["ax"], c["ay"], counts,
                                            2, f0=f0, workspace=ws)
        ms_f, _ = timed(fwd, est_steps, 2)
        ms_b, _ = timed(bwd, est_steps, 2)
        ms_vg, _ = timed(fused, est_steps, 2)
        s1, s5 = fwd()
        fa = fused()
        torch.cuda.synchronize()
        checks["albedo_lut"] = {"grid": g, "n": n, "s1": s1.cpu().numpy(),
                                "full_table": args.oracle_full_table,
                                "s5": s5.cpu().numpy(), "a004": fa[0].cpu().numpy(),
                                "g004": [x.cpu().numpy() for x in fa[1:]]}
        samples = 4096 * n
        out["albedo_lut"] = {
            "cells": 4096, "samples_per_cell": n, "timed_launches": est_steps,
            "fwd_bwd_ms": round(ms_vg, 4),
            "fwd_bwd_path": "albedo_value_and_grad: value and the three derivatives per cell in "
                            "one pass (what the autograd Function runs)",
            "fwd_ms": round(ms_f, 4), "bwd_ms": round(ms_b, 4),
            "separate_fwd_plus_bwd_ms": round(ms_f + ms_b, 4),
            "fwd_gsamples_per_s": round(samples / ms_f / 1e6, 2),
            "bwd_gsamples_per_s": round(samples / ms_b / 1e6, 2),
            "fwd_bwd_gsamples_per_s": round(samples / ms_vg / 1e6, 2),
            "roofline_fwd": alu_roofline("forward_two_sums", samples, ms_f),
            "roofline_fwd_bwd": alu_roofline("value_and_grad", samples, ms_vg)}
        if mix_ceiling:
            out["albedo_lut"]["frac_of_mix_ceiling"] = {
                "fwd": round(samples / ms_f / 1e6 / mix_ceiling["forward_two_sums"], 4),
                "fwd_bwd": round(samples / ms_vg / 1e6 / mix_ceiling["value_and_adjoint"], 4)}
        del c, ws
    if "grad" in only:
        log("differentiable albedo 32 x 32 x 2^18 through the autograd Function")
        gg = workloads.grad_grid(32, seed=3)
        ax = torch.from_numpy(gg["ax"]).to(dev).requires_grad_(True)
        ay = torch.from_numpy(gg["ay"]).to(dev).requires_grad_(True)
        th = torch.from_numpy(gg["theta"]).to(dev).requires_grad_(True)
        ph = torch.from_numpy(gg["phi"]).to(dev)
        f0 = torch.ones_like(ph)

        def fb():
            a = cv.albedo(ax, ay, th, ph, f0, 1 << 18, 3)
            a.sum().backward()
        ms_fb, _ = timed(fb, est_steps, 2)
        ms_f, _ = timed(lambda: cv.albedo(ax.detach(), ay.detach(), th.detach(), ph, f0,
                                          1 << 18, 3), est_steps, 2)
        out["albedo_grad"] = {"cells": 1024, "samples_per_cell": 1 << 18,
                              "timed_launches": est_steps,
                              "fwd_ms": round(ms_f, 4), "fwd_bwd_ms": round(ms_fb, 4)}
        # every cell, on the view directions the oracle's values were computed
        # on (rounded from double precision), through the one-pass kernel the
        # Function runs
        wx, wy, wz = workloads.view_from_angles(gg["theta"], gg["phi"])
        v = [torch.from_numpy(x).to(dev) for x in (wx, wy, wz, gg["ax"], gg["ay"])]
        r = cv.albedo_value_and_grad(*v, 1 << 18, 3)
        torch.cuda.synchronize()
        checks["albedo_grad"] = {"got": [x.cpu().numpy() for x in r]}
    if "batch" in only:
        log("batched estimator: 4096 uneven jobs, forward + adjoint (autotuned tiling)")
        j = workloads.batch_jobs(4096, seed=4)
        c = {k: torch.from_numpy(v).to(dev) for k, v in j.items() if k != "n"}
        t0 = time.perf_counter()
        best, best_ms = cv.albedo_batch_autotune(c["wx"], c["wy"], c["wz"], c["ax"], c["ay"],
                                                 j["n"], 4, with_grad=True)
        tune_s = time.perf_counter() - t0
        plan0 = cv.BatchPlan(c["wx"], c["wy"], c["wz"], c["ax"], c["ay"], j["n"], 4,
                             with_grad=True, tiling=(256, 32, 8, 0, 0))
        ms_default, _ = timed(plan0.run, est_steps, 2)
        plan0.close()
        plan0 = cv.BatchPlan(c["wx"], c["wy"], c["wz"], c["ax"], c["ay"], j["n"], 4,
                             with_grad=True, tiling=(256, 32, 8, 0, 1))
        ms_default_dyn, _ = timed(plan0.run, est_steps, 2)
        plan0.close()
        plan = cv.BatchPlan(c["wx"], c["wy"], c["wz"], c["ax"], c["ay"], j["n"], 4,
                            with_grad=True, tiling=best)
        outs_of = lambda: (plan.albedo, plan.grad_ax, plan.grad_ay, plan.grad_theta_o)  # noqa
        ms_b, _ = timed(plan.run, est_steps, 2)
        torch.cuda.synchronize()
        graph_out = [o.clone() for o in outs_of()]
        ms_r, _ = timed(plan.run_per_request, max(2, est_steps // 5), 1)
        torch.cuda.synchronize()
        req_out = [o.clone() for o in outs_of()]
        diff = {name: float(f"{(a - b).abs().max().item():.3e}") for name, a, b in
                zip(("albedo", "grad_ax", "grad_ay", "grad_theta_o"), graph_out, req_out)}
        checks["batched"] = {"graph": [x.cpu().numpy() for x in graph_out],
                             "per_request": [x.cpu().numpy() for x in req_out]}
        # The plain-sampler pipeline per request: fill the job's view and
        # roughness into reusable arrays, draw its uniforms (the estimator's
        # stream, so the samples are the batch's), run vndf_sample.  Such a
        # pipeline also needs a weighting and reduction pass, left out here,
        # so its time is a lower bound.  Timed eagerly and captured in one
        # graph (which removes the host's launch cost).
        plain_res = None
        if not args.no_plain_pipeline:
            log("per-request plain-sampler pipeline (lower bound: no weighting pass)")
            ns = [int(x) for x in j["n"]]
            nmax = max(ns)
            vals = [c[k].tolist() for k in ("wx", "wy", "wz", "ax", "ay")]
            bi = [torch.empty(nmax, device=dev) for _ in range(5)]
            bu = [torch.empty(nmax, device=dev) for _ in range(2)]
            bo = [torch.empty(nmax, device=dev) for _ in range(4)]

            def plain():
                for q, m in enumerate(ns):
                    for b, v in zip(bi, vals):
                        b[:m].fill_(v[q])
                    u1, u2 = cv.capvndf_uniforms(4, 3, q, 0, m, out=(bu[0][:m], bu[1][:m]))
                    cv.vndf_sample(bi[0][:m], bi[1][:m], bi[2][:m], bi[3][:m], bi[4][:m], u1=u1,
                                   u2=u2, method=HEADLINE_METHOD, out=tuple(o[:m] for o in bo))
            ms_plain, _ = timed(plain, 2, 1)
            t0 = time.perf_counter()
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph):
                plain()
            capture_s = time.perf_counter() - t0
            ms_plain_graph, _ = timed(graph.replay, 3, 1)
            del graph, bi, bu, bo
            plain_res = {"what": "per job: 5 fills, the job's uniforms, vndf_sample; no "
                                 "weighting or reduction pass (a lower bound)",
                         "eager_ms": round(ms_plain, 2),
                         "graph_ms": round(ms_plain_graph, 2),
                         "graph_capture_s": round(capture_s, 2),
                         "speedup_vs_graph": round(ms_plain_graph / ms_b, 2)}
        info = plan.info()
        out["batched"] = {"jobs": 4096, "total_samples": info["total_samples"],
                          "tiling": info["tiling"], "chunks": info["nchunks"],
                          "timed_launches": est_steps,
                          "graph_ms": round(ms_b, 4), "per_request_ms": round(ms_r, 4),
                          "speedup": round(ms_r / ms_b, 3),
                          "default_tiling_ms": round(ms_default, 4),
                          "default_tiling_dynamic_ms": round(ms_default_dyn, 4),
                          "autotune_s": round(tune_s, 2),
                          "gsamples_per_s_fwd_adj": round(info["total_samples"] / ms_b / 1e6, 2),
                          # over the whole replay (persistent kernel + finishing pass)
                          "roofline": alu_roofline(batch_kernel(info["tiling"]), info["total_samples"],
                                                   ms_b),
                          # the batch kernel's own counts are not in the summary;
                          # this prices its samples at the table's value +
                          # Jacobian kernel's count (the same per-sample code)
                          "roofline_proxy": proxy_roofline("value_and_grad", info["total_samples"],
                                                           ms_b),
                          "max_abs_diff_graph_vs_per_request": diff,
                          "per_request_plain_sampler": plain_res}
        plan.close()
        if not args.no_short_jobs:
            # a mix of short jobs (2^10 .. 2^14 samples), where wavefront-owned
            # chunks can beat block-owned ones: the autotuner decides
            log("batched estimator: 4096 short jobs (2^10 .. 2^14 samples), autotuned")
            js = workloads.batch_jobs(4096, seed=6, log2_min=10, log2_max=14)
            cs = {k: torch.from_numpy(v).to(dev) for k, v in js.items() if k != "n"}
            best_s, _ = cv.albedo_batch_autotune(cs["wx"], cs["wy"], cs["wz"], cs["ax"],
                                                 cs["ay"], js["n"], 4, with_grad=True)
            res_s = {}
            for name, til in (("autotuned", best_s), ("block_owned_default", (256, 32, 8, 0, 0)),
                              ("wave_owned", (256, 16, 8, 1, 0)),
                              ("wave_owned_dynamic", (256, 16, 8, 1, 1))):
                p2 = cv.BatchPlan(cs["wx"], cs["wy"], cs["wz"], cs["ax"], cs["ay"], js["n"], 4,
                                  with_grad=True, tiling=til)
                res_s[name + "_ms"] = round(timed(p2.run, max(MIN_EST_STEPS, args.steps // 5),
                                                  2)[0], 4)
                if name == "autotuned":
                    res_s["per_request_ms"] = round(timed(p2.run_per_request, 2, 1)[0], 4)
                    res_s["total_samples"] = p2.info()["total_samples"]
                p2.close()
            res_s["tiling"] = list(best_s)
            res_s["speedup_vs_per_request"] = round(res_s["per_request_ms"] /
                                                    res_s["autotuned_ms"], 2)
            out["batched"]["short_jobs"] = res_s

    if "radiance" in only:
        log("direct illumination 64 x 64 x 2^20 under 4 spherical-Gaussian lobes")
        g = workloads.lut_grid(64, 64)
        c = {k: torch.from_numpy(v).to(dev) for k, v in g.items()}
        n = 1 << 20
        counts = torch.full((4096,), n, dtype=torch.int64, device=dev)
        lobes_np = LOBES4
        lobes = torch.from_numpy(lobes_np).to(dev)
        ws = torch.empty(cv.albedo_workspace_size(4096, np.full(4096, n), 0) // 4 + 4,
                         device=dev)

        def rad():
            return cv.radiance_estimate(c["wx"], c["wy"], c["wz"], c["ax"], c["ay"], counts, 2,
                                        lobes, workspace=ws)
        ms_r, _ = timed(rad, est_steps, 2)
        r = rad()
        torch.cuda.synchronize()
        cells = np.array([5, 2900, 4095])
        r_all = r.cpu().numpy()
        checks["direct_illumination"] = {"grid": {k: v[cells] for k, v in g.items()},
                                         "cells": cells, "n": n, "lobes": lobes_np,
                                         "value": r_all[cells], "all": r_all}
        out["direct_illumination"] = {
            "cells": 4096, "samples_per_cell": n, "lobes": 4, "ms": round(ms_r, 4),
            "timed_launches": est_steps,
            "gsamples_per_s": round(4096 * n / ms_r / 1e6, 2),
            "roofline": alu_roofline("radiance", 4096 * n, ms_r)}
        if mix_ceiling:
            out["direct_illumination"]["frac_of_mix_ceiling"] = round(
                4096 * n / ms_r / 1e6 / mix_ceiling["radiance_4_lobes"], 4)

    result = {"metric": METRIC, "unit": "Gsamples/s", "n_gpus": 1, "steps": args.steps,
              "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
              "vs_baseline": None, "dtype": "f64", "data": "synthetic"}
    if ms_head is not None:
        achieved = BYTES_PER_SAMPLE * N_STREAM / (ms_head * 1e-3) / 1e9
        result["value"] = round(N_STREAM / ms_head / 1e6, 3)
        result["ms_per_step"] = round(ms_head, 5)
        result["wall_ms_per_step"] = round(wall_head, 5)
        result["launch_stats"] = head_stats
        result["settle_launches"] = SETTLE_LAUNCHES
        med = BYTES_PER_SAMPLE * N_STREAM / (head_stats["median_ms"] * 1e-3) / 1e9
        result["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1),
                              "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": round(achieved / HBM_PEAK_GBS, 4),
                              "traffic": measured_traffic(),
                              "frac_median_launch": round(med / HBM_PEAK_GBS, 4),
                              "trace": trace_figures()}
    else:
        result["value"] = None
        result["ms_per_step"] = None
    result["config"] = {
        "workload": "streaming anisotropic spherical-cap VNDF sampling: 2^26 tuples FP32 SoA, "
                    "cos(theta) in [1e-3, 1], alpha_x, alpha_y log-uniform in [1e-3, 1], "
                    "Philox uniforms in-kernel, outputs h and pdf",
        "tuples": N_STREAM, "method": "cap_f64",
        "arithmetic": "double precision from the FP32 inputs, outputs rounded to FP32 "
                      "(every h and pdf within 2e-6 of the exact sample)",
        "bytes_per_sample": BYTES_PER_SAMPLE, "parallelism": "single GPU"}
    result.update(out)
    if not args.no_cpu_baseline:
        if ms_head is not None:
            log("timing the FP64 oracle on the host's CPU share")
            result["cpu_baseline"] = cpu_baseline(d)
        if checks:
            log("checking the estimators against the FP64 oracle")
            for key, res in oracle_checks(checks).items():
                result[key].update(res)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
