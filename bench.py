"""Benchmark of the spherical-cap GGX VNDF hot path on one MI355X.

One step = one launch of the streaming cap sampler over 2^26 anisotropic
tuples (FP32 structure of arrays in HBM, Philox uniforms drawn in-kernel,
outputs h and its pdf).  The JSON line's value is that sampler's throughput in
Gsamples/s; alongside it the line reports the Heitz-2018 disk sampler on the
same inputs, the register-resident cap-vs-disk microbenchmark, the
directional-albedo table forward+backward time, the batched estimator against
per-request launches, the roofline of the streaming kernel, and -- in the CPU
leg, which is the only part that runs the FP64 oracle -- the oracle timed on
the host cores and its values at a few table cells, against which the
estimators' errors are reported.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--only SECTION ...]
           [--no-cpu-baseline]
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("Gsamples/s VNDF (cap vs 2018 disk) + albedo-LUT fwd+bwd time at "
          "≤1e-4 err")
N_STREAM = 1 << 26
BYTES_PER_SAMPLE = 36  # 5 FP32 inputs read + 4 FP32 outputs written
HBM_PEAK_GBS = 8000.0
SECTIONS = ("stream", "disk", "f64", "probe", "inverse", "dielectric", "micro", "lut", "grad",
            "batch", "radiance")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--only", nargs="*", default=None, choices=SECTIONS)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    return ap.parse_args()


def _bandwidth(bytes_per_element, ms):
    """GB/s of a streaming launch over the 2^26-element workload, and its
    fraction of the 8 TB/s HBM peak."""
    gbs = bytes_per_element * N_STREAM / ms / 1e6
    return {"gbytes_per_s": round(gbs, 1), "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}


def timed(fn, steps, warmup):
    """Mean ms per call of fn over `steps` calls on the current stream, with
    events recorded on that stream and device synchronisation around."""
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


def batch_kernel(tiling):
    """Counter-summary key of the batch kernel a tiling (block, pairs per
    thread, blocks per CU, per_wave, dynamic) runs, with gradients."""
    block, _, _, per_wave, dynamic = tiling
    name = "k_batch_wave" if per_wave else "k_batch"
    return f"batch:{name}<{block}, true, {'true' if dynamic else 'false'}>"


def cpu_baseline(d):
    """FP64 oracle on the host cores: the full 2^26-tuple workload of the
    streaming configuration (cap sampler + pdf, Philox uniforms)."""
    import numpy as np
    import oracle
    threads = min(os.cpu_count() or 1, 16)
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
            "kind": "oracle",
            "sample": f"all {n} tuples of the streaming workload, FP64 cap sampler + pdf; "
                      f"median of 3 runs ({dt:.2f} s each on {threads} host threads)"}


def oracle_checks(checks):
    """The CPU leg's second part: the FP64 oracle at the cells whose GPU values
    the estimator sections kept (same Philox streams): max |GPU - oracle| and
    the oracle's own throughput there (one host thread per cell)."""
    import numpy as np
    import oracle
    errs = {}
    threads = min(os.cpu_count() or 1, 16)
    if "albedo_lut" in checks:
        c = checks["albedo_lut"]
        g = c["grid"]
        wo = (g["wx"], g["wy"], g["wz"])
        t0 = time.perf_counter()
        a1 = oracle.albedo(wo, g["ax"], g["ay"], c["n"], 2, f0=1.0, units=c["cells"],
                           nthreads=threads)
        dt = time.perf_counter() - t0
        a5 = oracle.albedo(wo, g["ax"], g["ay"], c["n"], 2, f0=0.0, units=c["cells"],
                           nthreads=threads)
        err = max(np.abs(c["s1"] - a1).max(), np.abs(c["s5"] - a5).max(),
                  np.abs(c["a004"] - (0.04 * a1 + 0.96 * a5)).max())
        ns = len(c["cells"]) * c["n"]
        errs["albedo_lut"] = {
            "max_abs_err_vs_oracle": float(f"{err:.3e}"), "err_checked_cells": len(c["cells"]),
            "oracle": {"gsamples_per_s": round(ns / dt / 1e9, 6),
                       "cores": min(threads, len(c["cells"])),
                       "kind": "oracle", "sample": f"{len(c['cells'])} cells x {c['n']} "
                       f"samples, FP64 estimator, one Fresnel sum ({dt:.2f} s)"}}
    for key in ("albedo_grad", "batched"):
        if key not in checks:
            continue
        c = checks[key]
        t0 = time.perf_counter()
        ref = oracle.albedo_grad(c["wo"], c["ax"], c["ay"], c["n"], c["seed"], f0=1.0,
                                 units=c["units"], nthreads=threads)
        dt = time.perf_counter() - t0
        got = c["got"]
        e_val = float(np.abs(got[0] - ref[0]).max())
        ratio = max(float((np.abs(g_ - r_) / (1e-4 + 1e-3 * np.abs(r_))).max())
                    for g_, r_ in zip(got[1:], ref[1:]))
        ns = int(np.sum(np.broadcast_to(c["n"], (len(c["cells"]),))))
        errs[key] = {
            "max_abs_err_vs_oracle": float(f"{e_val:.3e}"),
            "max_grad_err_over_tolerance": round(ratio, 4),
            "grad_tolerance": "1e-4 + 1e-3 |g| against the oracle's dual-number gradient",
            "err_checked_cells": len(c["cells"]),
            "oracle": {"gsamples_per_s": round(ns / dt / 1e9, 6),
                       "cores": min(threads, len(c["cells"])),
                       "kind": "oracle", "sample": f"{len(c['cells'])} cells, {ns} samples, "
                       f"FP64 value + dual-number gradient ({dt:.2f} s)"}}
    if "direct_illumination" in checks:
        c = checks["direct_illumination"]
        g = c["grid"]
        ref = oracle.radiance((g["wx"], g["wy"], g["wz"]), g["ax"], g["ay"], c["n"], 2,
                              c["lobes"].astype(np.float64), units=c["cells"])
        errs["direct_illumination"] = {
            "max_abs_err_vs_oracle": float(f"{np.abs(c['value'] - ref).max():.3e}"),
            "err_checked_cells": len(c["cells"])}
    return errs


def main():
    args = parse()
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
    checks = {}  # GPU values at a few cells, compared with the oracle in the CPU leg

    log("generating the 2^26-tuple streaming workload")
    d = workloads.tuples_streaming(N_STREAM, seed=1)
    t = {k: torch.from_numpy(v).to(dev) for k, v in d.items()}
    outs = tuple(torch.empty_like(t["wx"]) for _ in range(4))

    def run(method):
        return lambda: cv.vndf_sample(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], seed=1,
                                      method=method, out=outs)

    ms_cap = wall_cap = None
    if "stream" in only:
        log("timing the cap sampler")
        ms_cap, wall_cap = timed(run(0), args.steps, args.warmup)
        log(f"cap: {ms_cap:.4f} ms/launch")
    if "disk" in only:
        log("timing the disk-2018 sampler")
        ms_disk, _ = timed(run(1), args.steps, args.warmup)
        out["disk2018"] = {"ms_per_launch": round(ms_disk, 5),
                           "gsamples_per_s": round(N_STREAM / ms_disk / 1e6, 3),
                           **_bandwidth(BYTES_PER_SAMPLE, ms_disk)}
        if ms_cap:
            out["disk2018"]["t_disk_over_t_cap"] = round(ms_disk / ms_cap, 4)
    if "f64" in only:
        log("timing the cap sampler in double precision")
        ms_f64, _ = timed(run(2), args.steps, args.warmup)
        out["cap_f64"] = {"what": "the same samples evaluated in double precision: every "
                                  "output within 2e-6 of the exact sample",
                          "ms_per_launch": round(ms_f64, 5),
                          "gsamples_per_s": round(N_STREAM / ms_f64 / 1e6, 3),
                          **_bandwidth(BYTES_PER_SAMPLE, ms_f64)}
        if ms_cap:
            out["cap_f64"]["t_f64_over_t_cap"] = round(ms_f64 / ms_cap, 4)
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
    if "inverse" in only:
        log("timing the inverse map h -> (u1, u2)")
        run(0)()
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
        # the methods alternate over several rounds, so that a drift of the
        # clock during the run moves all of them alike; medians are reported
        rounds = {name: [] for name, _ in methods}
        for _, m in methods:  # untimed: the first launches after a pause run on a cold clock
            timed(lambda: cv.vndf_microbench(m, lanes, iters, 1, out=buf), 50, 3)
        for _ in range(5):
            for name, m in methods:
                ms, _ = timed(lambda: cv.vndf_microbench(m, lanes, iters, 1, out=buf), 50, 3)
                rounds[name].append(ms)
        for name, _ in methods:
            ms = float(np.median(rounds[name]))
            res[name] = {"ms": round(ms, 5), "gsamples_per_s": round(lanes * iters / ms / 1e6, 2)}
        ratio = [d / c for d, c in zip(rounds["disk2018"], rounds["cap"])]
        res["t_disk_over_t_cap"] = round(float(np.median(ratio)), 4)
        res["t_disk_over_t_cap_rounds"] = [round(min(ratio), 4), round(max(ratio), 4)]
        # the double-precision cap's arithmetic without memory traffic to hide it
        res["t_cap_f64_over_t_cap"] = round(
            float(np.median([f / c for f, c in zip(rounds["cap_f64"], rounds["cap"])])), 4)
        res["lanes"] = lanes
        res["calls_per_lane"] = iters
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
        ws = torch.empty(cv.albedo_workspace_size(4096, n, 2) // 4 + 4, device=dev)
        f0 = torch.full((4096,), 0.04, device=dev)

        def fwd():
            return cv.albedo_estimate(c["wx"], c["wy"], c["wz"], c["ax"], c["ay"], n, 2,
                                      workspace=ws)

        def bwd():
            return cv.albedo_estimate_backward(c["wx"], c["wy"], c["wz"], c["ax"], c["ay"], n, 2,
                                               workspace=ws)

        def fused():
            return cv.albedo_value_and_grad(c["wx"], c["wy"], c["wz"], c["ax"], c["ay"], n, 2,
                                            f0=f0, workspace=ws)
        steps = max(3, args.steps // 10)
        ms_f, _ = timed(fwd, steps, 2)
        ms_b, _ = timed(bwd, steps, 2)
        ms_vg, _ = timed(fused, steps, 2)
        s1, s5 = fwd()
        a004 = fused()[0]
        torch.cuda.synchronize()
        cells = np.linspace(0, 4095, 16).astype(np.int64)
        checks["albedo_lut"] = {"grid": {k: v[cells] for k, v in g.items()}, "cells": cells,
                                "n": n, "s1": s1.cpu().numpy()[cells],
                                "s5": s5.cpu().numpy()[cells],
                                "a004": a004.cpu().numpy()[cells]}
        samples = 4096 * n
        out["albedo_lut"] = {
            "cells": 4096, "samples_per_cell": n,
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
        ms_fb, _ = timed(fb, max(3, args.steps // 10), 2)
        ms_f, _ = timed(lambda: cv.albedo(ax.detach(), ay.detach(), th.detach(), ph, f0,
                                          1 << 18, 3), max(3, args.steps // 10), 2)
        out["albedo_grad"] = {"cells": 1024, "samples_per_cell": 1 << 18,
                              "fwd_ms": round(ms_f, 4), "fwd_bwd_ms": round(ms_fb, 4)}
        # one clean pass for the oracle comparison in the CPU leg
        for p_ in (ax, ay, th):
            p_.grad = None
        a = cv.albedo(ax, ay, th, ph, f0, 1 << 18, 3)
        a.sum().backward()
        with torch.no_grad():
            st = torch.sin(th)
            wo = (st * torch.cos(ph), st * torch.sin(ph), torch.cos(th))
        torch.cuda.synchronize()
        cells = np.linspace(0, 1023, 16).astype(np.int64)
        checks["albedo_grad"] = {
            "wo": tuple(x.detach().cpu().numpy()[cells] for x in wo),
            "ax": gg["ax"][cells], "ay": gg["ay"][cells], "n": 1 << 18, "seed": 3,
            "cells": cells, "units": cells,
            "got": [x.detach().cpu().numpy()[cells] for x in (a, ax.grad, ay.grad, th.grad)]}
    if "batch" in only:
        log("batched estimator: 4096 uneven jobs, forward + adjoint (autotuned tiling)")
        j = workloads.batch_jobs(4096, seed=4)
        c = {k: torch.from_numpy(v).to(dev) for k, v in j.items() if k != "n"}
        t0 = time.perf_counter()
        best, best_ms = cv.albedo_batch_autotune(c["wx"], c["wy"], c["wz"], c["ax"], c["ay"],
                                                 j["n"], 4, with_grad=True)
        tune_s = time.perf_counter() - t0
        steps = max(3, args.steps // 10)
        plan0 = cv.BatchPlan(c["wx"], c["wy"], c["wz"], c["ax"], c["ay"], j["n"], 4,
                             with_grad=True, tiling=(256, 32, 8, 0, 0))
        ms_default, _ = timed(plan0.run, steps, 2)
        plan0.close()
        plan0 = cv.BatchPlan(c["wx"], c["wy"], c["wz"], c["ax"], c["ay"], j["n"], 4,
                             with_grad=True, tiling=(256, 32, 8, 0, 1))
        ms_default_dyn, _ = timed(plan0.run, steps, 2)
        plan0.close()
        plan = cv.BatchPlan(c["wx"], c["wy"], c["wz"], c["ax"], c["ay"], j["n"], 4,
                            with_grad=True, tiling=best)
        ms_b, _ = timed(plan.run, steps, 2)
        ref = [o.clone() for o in (plan.albedo, plan.grad_ax)]
        ms_r, _ = timed(plan.run_per_request, max(2, steps // 2), 1)
        dev_a = (plan.albedo - ref[0]).abs().max().item()
        # 256 jobs drawn from all 4096 (every size), value and gradients
        jobs = np.sort(np.random.default_rng(0).choice(len(j["n"]), 256, replace=False))
        checks["batched"] = {
            "wo": tuple(j[k][jobs] for k in ("wx", "wy", "wz")), "ax": j["ax"][jobs],
            "ay": j["ay"][jobs], "n": j["n"][jobs], "seed": 4, "cells": jobs, "units": jobs,
            "got": [x.cpu().numpy()[jobs] for x in (plan.albedo, plan.grad_ax, plan.grad_ay,
                                                    plan.grad_theta_o)]}
        # The plain-sampler pipeline per request: fill the job's view and
        # roughness into reusable arrays, draw its uniforms (the estimator's
        # stream, so the samples are the batch's), run vndf_sample.  Such a
        # pipeline also needs a weighting and reduction pass, left out here,
        # so its time is a lower bound.  Timed eagerly and captured in one
        # graph (which removes the host's launch cost).
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
                               u2=u2, out=tuple(o[:m] for o in bo))
        ms_plain, _ = timed(plain, 2, 1)
        t0 = time.perf_counter()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            plain()
        capture_s = time.perf_counter() - t0
        ms_plain_graph, _ = timed(graph.replay, 3, 1)
        del graph, bi, bu, bo
        info = plan.info()
        out["batched"] = {"jobs": 4096, "total_samples": info["total_samples"],
                          "tiling": info["tiling"], "chunks": info["nchunks"],
                          "graph_ms": round(ms_b, 4), "per_request_ms": round(ms_r, 4),
                          "speedup": round(ms_r / ms_b, 3),
                          "default_tiling_ms": round(ms_default, 4),
                          "default_tiling_dynamic_ms": round(ms_default_dyn, 4),
                          "autotune_s": round(tune_s, 2),
                          "gsamples_per_s_fwd_adj": round(info["total_samples"] / ms_b / 1e6, 2),
                          # over the whole replay (persistent kernel + finishing pass)
                          "roofline": alu_roofline(batch_kernel(info["tiling"]), info["total_samples"],
                                                   ms_b),
                          "max_abs_albedo_diff_batch_vs_per_request": float(f"{dev_a:.3e}"),
                          "per_request_plain_sampler": {
                              "what": "per job: 5 fills, the job's uniforms, vndf_sample; no "
                                      "weighting or reduction pass (a lower bound)",
                              "eager_ms": round(ms_plain, 2),
                              "graph_ms": round(ms_plain_graph, 2),
                              "graph_capture_s": round(capture_s, 2),
                              "speedup_vs_graph": round(ms_plain_graph / ms_b, 2)}}
        plan.close()
        # a mix of short jobs (2^10 .. 2^14 samples), where wavefront-owned
        # chunks can beat block-owned ones: the autotuner decides
        log("batched estimator: 4096 short jobs (2^10 .. 2^14 samples), autotuned")
        js = workloads.batch_jobs(4096, seed=6, log2_min=10, log2_max=14)
        cs = {k: torch.from_numpy(v).to(dev) for k, v in js.items() if k != "n"}
        best_s, _ = cv.albedo_batch_autotune(cs["wx"], cs["wy"], cs["wz"], cs["ax"], cs["ay"],
                                             js["n"], 4, with_grad=True)
        res_s = {}
        for name, til in (("autotuned", best_s), ("block_owned_default", (256, 32, 8, 0, 0)),
                          ("wave_owned", (256, 16, 8, 1, 0)),
                          ("wave_owned_dynamic", (256, 16, 8, 1, 1))):
            p2 = cv.BatchPlan(cs["wx"], cs["wy"], cs["wz"], cs["ax"], cs["ay"], js["n"], 4,
                              with_grad=True, tiling=til)
            res_s[name + "_ms"] = round(timed(p2.run, max(5, args.steps // 5), 2)[0], 4)
            if name == "autotuned":
                res_s["per_request_ms"] = round(timed(p2.run_per_request, 2, 1)[0], 4)
                res_s["total_samples"] = p2.info()["total_samples"]
            p2.close()
        res_s["tiling"] = list(best_s)
        res_s["speedup_vs_per_request"] = round(res_s["per_request_ms"] / res_s["autotuned_ms"], 2)
        out["batched"]["short_jobs"] = res_s

    if "radiance" in only:
        log("direct illumination 64 x 64 x 2^20 under 4 spherical-Gaussian lobes")
        g = workloads.lut_grid(64, 64)
        c = {k: torch.from_numpy(v).to(dev) for k, v in g.items()}
        n = 1 << 20
        lobes_np = np.array([[0.0, 0.0, 1.0, 4.0, 2.0], [0.6, 0.0, 0.8, 30.0, 5.0],
                             [-0.5, 0.5, 0.70710678, 10.0, 1.5], [0.0, 0.0, 1.0, 0.0, 0.3]],
                            dtype=np.float32)
        lobes = torch.from_numpy(lobes_np).to(dev)
        ws = torch.empty(cv.albedo_workspace_size(4096, n, 0) // 4 + 4, device=dev)

        def rad():
            return cv.radiance_estimate(c["wx"], c["wy"], c["wz"], c["ax"], c["ay"], n, 2, lobes,
                                        workspace=ws)
        ms_r, _ = timed(rad, max(3, args.steps // 10), 2)
        r = rad()
        torch.cuda.synchronize()
        cells = np.array([5, 2900, 4095])
        checks["direct_illumination"] = {"grid": {k: v[cells] for k, v in g.items()},
                                         "cells": cells, "n": n, "lobes": lobes_np,
                                         "value": r.cpu().numpy()[cells]}
        out["direct_illumination"] = {
            "cells": 4096, "samples_per_cell": n, "lobes": 4, "ms": round(ms_r, 4),
            "gsamples_per_s": round(4096 * n / ms_r / 1e6, 2),
            "roofline": alu_roofline("radiance", 4096 * n, ms_r)}

    result = {"metric": METRIC, "unit": "Gsamples/s", "n_gpus": 1, "steps": args.steps,
              "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
              "vs_baseline": None, "dtype": "f32", "data": "synthetic"}
    if ms_cap is not None:
        achieved = BYTES_PER_SAMPLE * N_STREAM / (ms_cap * 1e-3) / 1e9
        result["value"] = round(N_STREAM / ms_cap / 1e6, 3)
        result["ms_per_step"] = round(ms_cap, 5)
        result["wall_ms_per_step"] = round(wall_cap, 5)
        result["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1),
                              "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": round(achieved / HBM_PEAK_GBS, 4),
                              "traffic": measured_traffic()}
    else:
        result["value"] = None
        result["ms_per_step"] = None
    result["config"] = {
        "workload": "streaming anisotropic spherical-cap VNDF sampling: 2^26 tuples FP32 SoA, "
                    "cos(theta) in [1e-3, 1], alpha_x, alpha_y log-uniform in [1e-3, 1], "
                    "Philox uniforms in-kernel, outputs h and pdf",
        "tuples": N_STREAM, "method": "cap", "bytes_per_sample": BYTES_PER_SAMPLE,
        "parallelism": "single GPU"}
    result.update(out)
    if not args.no_cpu_baseline:
        if ms_cap is not None:
            log("timing the FP64 oracle on the host cores")
            result["cpu_baseline"] = cpu_baseline(d)
        if checks:
            log("checking the estimators at sampled cells against the FP64 oracle")
            for key, res in oracle_checks(checks).items():
                result[key].update(res)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
