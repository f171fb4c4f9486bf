"""Pins of the oracle's horizon-band bound (CPU only).

oracle.albedo_horizon_band bounds how much the estimator's gradient can move
when the samples whose reflected direction lies within a band around the
horizon change side.  The pin moves them for real: a copy of the oracle whose
horizon test sits at wb_z = eps instead of 0 kills every sample with
0 < wb_z <= eps, and the change of its dual-number gradient must stay within
the bound computed for the band |wb_z| <= eps -- and reach about the bound
where a single sample lies in the band."""

import ctypes
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.cpp")
EPS = 1e-4
SITE = "if (!(value(wb.z) > 0.0)) return T(0.0);"


@pytest.fixture(scope="module")
def shifted(tmp_path_factory):
    src = open(SRC).read()
    assert src.count(SITE) == 1
    d = tmp_path_factory.mktemp("shifted")
    with open(d / "oracle.cpp", "w") as f:
        f.write(src.replace(SITE, f"if (!(value(wb.z) > {EPS!r})) return T(0.0);"))
    lib = str(d / "liboracle.so")
    subprocess.run(["g++", "-O2", "-std=gnu++17", "-fPIC", "-shared", "-pthread",
                    "-ffp-contract=off", str(d / "oracle.cpp"), "-o", lib, "-lquadmath"],
                   check=True)
    return lib


def _grad_with(lib, j, n):
    code = ("import sys, numpy as np; sys.path.insert(0, %r); import oracle, workloads\n"
            "j = workloads.batch_jobs(64, seed=4, log2_min=14, log2_max=14)\n"
            "r = oracle.albedo_grad((j['wx'], j['wy'], j['wz']), j['ax'], j['ay'], %d, 4)\n"
            "np.save(sys.argv[1], np.stack(r))\n") % (ROOT, n)
    out = lib + ".npy"
    env = dict(os.environ, CAPVNDF_ORACLE_LIB=lib)
    subprocess.run([sys.executable, "-c", code, out], check=True, env=env, cwd=ROOT)
    return np.load(out)


def test_band_bounds_a_real_change_of_side(shifted):
    n = 1 << 14
    j = workloads.batch_jobs(64, seed=4, log2_min=14, log2_max=14)
    wo = (j["wx"], j["wy"], j["wz"])
    base = np.stack(oracle.albedo_grad(wo, j["ax"], j["ay"], n, 4))
    moved = _grad_with(shifted, j, n)
    bx, by, bt, cnt = oracle.albedo_horizon_band(wo, j["ax"], j["ay"], n, 4,
                                                 c0=EPS * 2.0 ** 24, c1=0.0)
    assert np.abs(moved[0] - base[0]).max() < 1e-4  # the weight is continuous there
    hit = 0
    for k, b in enumerate((bx, by, bt)):
        diff = np.abs(moved[k + 1] - base[k + 1])
        assert np.all(diff <= b * (1 + 1e-9) + 1e-15), (k, np.max(diff - b))
        assert np.all(diff[cnt == 0] <= 1e-15)
        # a single sample in the band: the bound is its own slope jump; the
        # killed side (0, eps] is half the band, so about half the single
        # samples moved by about their bound
        one = (cnt == 1) & (b > 1e-9)
        close = np.abs(diff[one] - b[one]) <= 0.05 * b[one]
        hit += int(close.sum())
    print(f"jobs with samples in the band: {int((cnt > 0).sum())} of 64, "
          f"single-sample bounds met within 5 %: {hit}")
    assert (cnt > 0).sum() >= 3 and hit >= 1


def test_band_is_empty_without_width():
    j = workloads.batch_jobs(16, seed=4, log2_min=12, log2_max=12)
    r = oracle.albedo_horizon_band((j["wx"], j["wy"], j["wz"]), j["ax"], j["ay"], 4096, 4,
                                   c0=0.0, c1=0.0)
    assert np.all(r[3] == 0) and all(np.all(x == 0) for x in r[:3])
