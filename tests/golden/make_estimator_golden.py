"""Writes the FP64 oracle's values for every unit of the three estimator
workloads into ``estimator_full.npz`` next to this script.

Only the oracle (``oracle/``) and the seeded input generators
(``workloads.py``) are called; nothing here touches the GPU library.  The GPU
parity tests read the file and compare the library's output for every cell
and job against it, so the full-size comparison costs the tests seconds
instead of the oracle's minutes.

Workloads (the estimator of Appendix A with L == 1 on the Philox streams of
tag 3, unit = cell or job index):

* ``lut``   -- the 64 x 64 directional-albedo table, 2^20 samples per cell,
  seed 2: the two sums S1 (F0 = 1) and S5 (F0 = 0), and the value with its
  three dual-number derivatives (alpha_x, alpha_y, theta_o) at F0 = 0.04.
* ``grad``  -- the 32 x 32 anisotropic gradient grid, 2^18 samples per cell,
  seed 3, F0 = 1: value, the three dual-number derivatives, and central
  differences of the same estimator with step 1e-4.
* ``batch`` -- the 4096 uneven jobs (2^10 .. 2^22 samples), seed 4, F0 = 1:
  value and the three dual-number derivatives.
* ``radiance`` -- direct illumination over the same 64 x 64 table, 2^20
  samples per cell, seed 2, F0 = 1, under four spherical-Gaussian lobes
  (RAD_LOBES, the benchmark's): the estimator of Appendix A with the lobes'
  radiance L(w_l) in place of L == 1.

For each workload the file also holds, per cell or job, the oracle's bound on
how far the gradient may move when samples whose reflected direction lies
within rounding of the horizon land on the other side
(oracle.albedo_horizon_band): the GPU kernels evaluate every sample whose
FP32 reflection is that close to the horizon again in double precision, so
the band is the double-precision one, (44 + 192 kappa) 2^-48; the parity
tests add its bound to the gradient tolerance.

The table's S1 pass runs through the oracle's own all-core path and is timed
(the "full table once" figure); the other passes are scheduled one unit per
call over a thread pool, longest first, because the job sizes are uneven.
The file also records a digest of every input array, the wall times, the
thread count and the host's CPU model.

Usage: python tests/golden/make_estimator_golden.py [--threads T]
           [--only lut grad batch bands radiance]
"""

from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

OUT = os.path.join(HERE, "estimator_full.npz")

LUT_N, LUT_SEED, LUT_F0 = 1 << 20, 2, 0.04
GRAD_N, GRAD_SEED, GRAD_STEP = 1 << 18, 3, 1e-4
BATCH_SEED = 4
RAD_N, RAD_SEED = 1 << 20, 2
# rows (mu_x, mu_y, mu_z, kappa, lambda), float32 as the library receives them
RAD_LOBES = np.array([[0.0, 0.0, 1.0, 4.0, 2.0], [0.6, 0.0, 0.8, 30.0, 5.0],
                      [-0.5, 0.5, 0.70710678, 10.0, 1.5], [0.0, 0.0, 1.0, 0.0, 0.3]],
                     dtype=np.float32)
# the kernels' double-precision horizon decision: band (c0 + c1 kappa) 2^-48
BAND_C0, BAND_C1 = oracle.HORIZON_C0 * 2.0 ** -24, oracle.HORIZON_C1 * 2.0 ** -24


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def digest(arrays: dict) -> str:
    h = hashlib.sha256()
    for k in sorted(arrays):
        a = np.ascontiguousarray(arrays[k])
        h.update(k.encode())
        h.update(str(a.dtype).encode())
        h.update(a.tobytes())
    return h.hexdigest()[:32]


def lut_inputs():
    return workloads.lut_grid(64, 64)


def grad_inputs():
    gg = workloads.grad_grid(32, seed=GRAD_SEED)
    wx, wy, wz = workloads.view_from_angles(gg["theta"], gg["phi"])
    return {"wx": wx, "wy": wy, "wz": wz, "ax": gg["ax"], "ay": gg["ay"]}


def batch_inputs():
    return workloads.batch_jobs(4096, seed=BATCH_SEED)


def radiance_inputs():
    return {**workloads.lut_grid(64, 64), "lobes": RAD_LOBES}


def per_unit(fn, g, n, seed, threads, nout, **kw):
    """fn over every unit, one unit per call (nthreads=1) on a thread pool,
    largest sample count first; returns nout arrays indexed by unit."""
    units = g["wx"].shape[0]
    ns = np.broadcast_to(np.asarray(n, dtype=np.int64), (units,))
    order = np.argsort(-ns, kind="stable")
    outs = [np.zeros(units) for _ in range(nout)]

    def one(i):
        sub = (g["wx"][i:i + 1], g["wy"][i:i + 1], g["wz"][i:i + 1])
        r = fn(sub, g["ax"][i:i + 1], g["ay"][i:i + 1], ns[i:i + 1], seed, units=[i],
               nthreads=1, **kw)
        return i, (r,) if nout == 1 else r

    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        for i, r in ex.map(one, order):
            for k in range(nout):
                outs[k][i] = r[k][0]
    return outs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--only", nargs="*", default=["lut", "grad", "batch", "bands", "radiance"])
    args = ap.parse_args()
    T = args.threads
    rec = {}
    if os.path.exists(OUT):
        with np.load(OUT, allow_pickle=False) as f:
            rec = {k: f[k] for k in f.files}
    rec["host_cpu_model"] = np.array(cpu_model())
    rec["host_threads"] = np.array(T)

    if "lut" in args.only:
        g = lut_inputs()
        wo = (g["wx"], g["wy"], g["wz"])
        t0 = time.perf_counter()
        s1 = oracle.albedo(wo, g["ax"], g["ay"], LUT_N, LUT_SEED, f0=1.0, nthreads=T)
        t_s1 = time.perf_counter() - t0
        print(f"lut S1: {t_s1:.1f} s on {T} threads "
              f"({4096 * LUT_N / t_s1 / 1e9:.3f} Gsamples/s)", flush=True)
        t0 = time.perf_counter()
        s5 = oracle.albedo(wo, g["ax"], g["ay"], LUT_N, LUT_SEED, f0=0.0, nthreads=T)
        print(f"lut S5: {time.perf_counter() - t0:.1f} s", flush=True)
        t0 = time.perf_counter()
        a, gx, gy, gt = per_unit(oracle.albedo_grad, g, LUT_N, LUT_SEED, T, 4, f0=LUT_F0)
        t_g = time.perf_counter() - t0
        print(f"lut value + gradient: {t_g:.1f} s", flush=True)
        rec.update({"lut_digest": np.array(digest(g)), "lut_n": np.array(LUT_N),
                    "lut_seed": np.array(LUT_SEED), "lut_f0": np.array(LUT_F0),
                    "lut_s1": s1, "lut_s5": s5, "lut_value": a, "lut_gax": gx, "lut_gay": gy,
                    "lut_gth": gt, "lut_s1_seconds": np.array(t_s1),
                    "lut_grad_seconds": np.array(t_g)})

    if "grad" in args.only:
        g = grad_inputs()
        t0 = time.perf_counter()
        a, gx, gy, gt = per_unit(oracle.albedo_grad, g, GRAD_N, GRAD_SEED, T, 4, f0=1.0)
        fx, fy, ft = per_unit(oracle.albedo_fd, g, GRAD_N, GRAD_SEED, T, 3, f0=1.0,
                              step=GRAD_STEP)
        print(f"grad grid: {time.perf_counter() - t0:.1f} s", flush=True)
        rec.update({"grad_digest": np.array(digest(g)), "grad_n": np.array(GRAD_N),
                    "grad_seed": np.array(GRAD_SEED), "grad_value": a, "grad_gax": gx,
                    "grad_gay": gy, "grad_gth": gt, "grad_fd_step": np.array(GRAD_STEP),
                    "grad_fd_ax": fx, "grad_fd_ay": fy, "grad_fd_th": ft})

    if "batch" in args.only:
        j = batch_inputs()
        t0 = time.perf_counter()
        a, gx, gy, gt = per_unit(oracle.albedo_grad, j, j["n"], BATCH_SEED, T, 4, f0=1.0)
        t_b = time.perf_counter() - t0
        print(f"batch: {t_b:.1f} s ({int(j['n'].sum())} samples)", flush=True)
        rec.update({"batch_digest": np.array(digest(j)), "batch_seed": np.array(BATCH_SEED),
                    "batch_n": j["n"], "batch_value": a, "batch_gax": gx, "batch_gay": gy,
                    "batch_gth": gt, "batch_seconds": np.array(t_b)})

    if "bands" in args.only:
        t0 = time.perf_counter()
        for part, inputs, n, seed, f0 in (("lut", lut_inputs(), LUT_N, LUT_SEED, LUT_F0),
                                          ("grad", grad_inputs(), GRAD_N, GRAD_SEED, 1.0),
                                          ("batch", batch_inputs(), None, BATCH_SEED, 1.0)):
            counts = inputs["n"] if n is None else n
            bx, by, bt, bc = per_unit(oracle.albedo_horizon_band, inputs, counts, seed, T, 4,
                                      f0=f0, c0=BAND_C0, c1=BAND_C1)
            rec.update({f"{part}_band_ax": bx, f"{part}_band_ay": by, f"{part}_band_th": bt,
                        f"{part}_band_count": bc.astype(np.int64),
                        "band_c0": np.array(BAND_C0), "band_c1": np.array(BAND_C1)})
        print(f"horizon bands: {time.perf_counter() - t0:.1f} s", flush=True)

    if "radiance" in args.only:
        g = radiance_inputs()
        t0 = time.perf_counter()
        r = oracle.radiance((g["wx"], g["wy"], g["wz"]), g["ax"], g["ay"], RAD_N, RAD_SEED,
                            RAD_LOBES.astype(np.float64), f0=1.0, nthreads=T)
        t_r = time.perf_counter() - t0
        print(f"radiance: {t_r:.1f} s", flush=True)
        rec.update({"radiance_digest": np.array(digest(g)), "radiance_n": np.array(RAD_N),
                    "radiance_seed": np.array(RAD_SEED), "radiance_lobes": RAD_LOBES,
                    "radiance_value": r, "radiance_seconds": np.array(t_r)})

    np.savez_compressed(OUT, **rec)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
