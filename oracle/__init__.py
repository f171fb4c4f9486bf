"""FP64 CPU oracle for spherical-cap GGX VNDF sampling (arXiv 2306.05044).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference the GPU library is checked against.  Only the test suite, the smoke
check and the CPU-baseline leg of the benchmark may import it.  It shares no
code with the HIP library and never loads it.

The arithmetic lives in ``oracle.cpp`` (C++17, double precision, no fast-math);
this module builds it with g++ and wraps its C entry points for numpy arrays.
Each wrapper names the passage of the paper it follows; see the header of
``oracle.cpp`` for the readings taken where the paper is silent.

Functions whose result has no pin other than the oracle itself say so here:
none at present (every routine is pinned by a test in ``tests/test_oracle_*``).
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
# A test may point the wrapper at another build of the oracle (the mutation
# test builds deliberately broken copies and checks that the pins fail).
_LIB_OVERRIDE = os.environ.get("CAPVNDF_ORACLE_LIB")
# Thread count used when a call passes nthreads=0 (0 = all hardware threads).
_THREADS = int(os.environ.get("CAPVNDF_ORACLE_THREADS", "0"))

TAG_SAMPLE = 2
TAG_ALBEDO = 3
TAG_DIELECTRIC = 5
CAP = 0
DISK2018 = 1


def build() -> str:
    """Compile ``oracle.cpp`` into ``liboracle.so`` (always recompiles)."""
    cmd = [
        "g++", "-O2", "-std=gnu++17", "-fPIC", "-shared", "-pthread",
        "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
        _SRC, "-o", _LIB + ".tmp", "-lquadmath",
    ]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None

_d = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.POINTER(ctypes.c_int64)
_u32 = ctypes.POINTER(ctypes.c_uint32)
_i32 = ctypes.POINTER(ctypes.c_int32)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if _LIB_OVERRIDE:
        lib = ctypes.CDLL(_LIB_OVERRIDE)
    else:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
    lib.orc_philox4x32_10.argtypes = [_u32, _u32, _u32]
    lib.orc_philox4x32_10.restype = None
    lib.orc_uniforms.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                 ctypes.c_uint64, ctypes.c_int64, _d, _d]
    lib.orc_uniforms.restype = None
    lib.orc_hemisphere_sample.argtypes = [ctypes.c_int64, _d, _d, _d, _d, _d,
                                          ctypes.c_int32, _d, _d, _d]
    lib.orc_hemisphere_sample.restype = None
    lib.orc_vndf_sample.argtypes = [ctypes.c_int64, _d, _d, _d, _d, _d, _d, _d,
                                    ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int32,
                                    _d, _d, _d, _d, ctypes.c_int32]
    lib.orc_vndf_sample.restype = ctypes.c_int32
    lib.orc_vndf_pdf.argtypes = [ctypes.c_int64, _d, _d, _d, _d, _d, _d, _d, _d, _d,
                                 ctypes.c_int32]
    lib.orc_vndf_pdf.restype = ctypes.c_int32
    lib.orc_ggx_ndf.argtypes = [ctypes.c_int64, _d, _d, _d, _d, _d, _d]
    lib.orc_ggx_ndf.restype = None
    lib.orc_smith_g1.argtypes = [ctypes.c_int64, _d, _d, _d, _d, _d, _d, _d, _d, _d]
    lib.orc_smith_g1.restype = None
    lib.orc_brdf.argtypes = [ctypes.c_int64, _d, _d, _d, _d, _d, _d, _d, _d,
                             ctypes.c_double, _d]
    lib.orc_brdf.restype = None
    lib.orc_albedo_terms.argtypes = [ctypes.c_int64, _d, _d, _d, _d, _d, _d, _d,
                                     ctypes.c_double, ctypes.c_int32, _d]
    lib.orc_albedo_terms.restype = None
    lib.orc_albedo.argtypes = [ctypes.c_int64, _d, _d, _d, _d, _d, _i64, _u32,
                               ctypes.c_uint64, _d, ctypes.c_int32, _d, ctypes.c_int32]
    lib.orc_albedo.restype = ctypes.c_int32
    lib.orc_albedo_grad.argtypes = [ctypes.c_int64, _d, _d, _d, _d, _d, _i64, _u32,
                                    ctypes.c_uint64, _d, _d, _d, _d, _d, ctypes.c_int32]
    lib.orc_albedo_grad.restype = ctypes.c_int32
    lib.orc_albedo_fd.argtypes = [ctypes.c_int64, _d, _d, _d, _d, _d, _i64, _u32,
                                  ctypes.c_uint64, _d, ctypes.c_double, _d, _d, _d,
                                  ctypes.c_int32]
    lib.orc_albedo_fd.restype = ctypes.c_int32
    lib.orc_albedo_kinks.argtypes = [ctypes.c_int64, _d, _d, _d, _d, _d, _i64, _u32,
                                     ctypes.c_uint64, ctypes.c_double, _i64, _i64, _i64,
                                     ctypes.c_int32]
    lib.orc_albedo_kinks.restype = ctypes.c_int32
    lib.orc_albedo_horizon_band.argtypes = [ctypes.c_int64, _d, _d, _d, _d, _d, _i64, _u32,
                                            ctypes.c_uint64, _d, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_double, _d, _d, _d, _i64,
                                            ctypes.c_int32]
    lib.orc_albedo_horizon_band.restype = ctypes.c_int32
    lib.orc_radiance.argtypes = [ctypes.c_int64, _d, _d, _d, _d, _d, _d, _i64, _u32,
                                 ctypes.c_uint64, _d, ctypes.c_int32, _d, ctypes.c_int32]
    lib.orc_radiance.restype = ctypes.c_int32
    lib.orc_radiance_at.argtypes = [ctypes.c_int64, _d, _d, _d, _d, ctypes.c_int32, _d]
    lib.orc_radiance_at.restype = None
    lib.orc_vndf_inverse.argtypes = [ctypes.c_int64, _d, _d, _d, _d, _d, _d, _d, _d, _d, _d,
                                     ctypes.c_int32]
    lib.orc_vndf_inverse.restype = ctypes.c_int32
    lib.orc_dielectric_sample.argtypes = [ctypes.c_int64, _d, _d, _d, _d, _d, ctypes.c_double,
                                          _d, _d, _d, ctypes.c_uint64, ctypes.c_uint64,
                                          _d, _d, _d, _d, _d, _i32, _d, _d, _d, ctypes.c_int32]
    lib.orc_dielectric_sample.restype = ctypes.c_int32
    lib.orc_dielectric_eval.argtypes = [ctypes.c_int64, _d, _d, _d, _d, _d, _d, _d, _d,
                                        ctypes.c_double, _d, _d, ctypes.c_int32]
    lib.orc_dielectric_eval.restype = ctypes.c_int32
    lib.orc_fresnel_dielectric.argtypes = [ctypes.c_int64, _d, ctypes.c_double, _d]
    lib.orc_fresnel_dielectric.restype = None
    lib.orc_dielectric_uniforms.argtypes = [ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64,
                                            _d, _d, _d]
    lib.orc_dielectric_uniforms.restype = None
    lib.orc_hardware_threads.argtypes = []
    lib.orc_hardware_threads.restype = ctypes.c_int32
    _lib = lib
    return lib


def _f64(a, n=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if n is not None:
        a = np.broadcast_to(a, (n,)).copy() if a.ndim == 0 or a.shape != (n,) else a
    return a


def _nt(nthreads):
    return nthreads if nthreads else _THREADS


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(_d)


def hardware_threads() -> int:
    return int(_load().orc_hardware_threads())


def philox4x32_10(ctr, key) -> np.ndarray:
    """Philox4x32-10 block (Salmon et al., SC'11): four 32-bit output words."""
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32).reshape(4))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32).reshape(2))
    out = np.zeros(4, dtype=np.uint32)
    _load().orc_philox4x32_10(c.ctypes.data_as(_u32), k.ctypes.data_as(_u32),
                              out.ctypes.data_as(_u32))
    return out


def uniforms(seed: int, tag: int, unit: int, k0: int, n: int):
    """(u1, u2) of samples k0..k0+n-1 of stream (seed, tag, unit)."""
    u1 = np.zeros(n)
    u2 = np.zeros(n)
    _load().orc_uniforms(seed, tag, unit, k0, n, _p(u1), _p(u2))
    return u1, u2


def hemisphere_sample(wi, u1, u2, method=CAP):
    """Hemisphere sampler of Sec. 3.3 (cap) or Sec. 2 (disk), unnormalised."""
    wi = [_f64(c) for c in wi]
    n = wi[0].shape[0]
    u1 = _f64(u1, n)
    u2 = _f64(u2, n)
    h = [np.zeros(n) for _ in range(3)]
    _load().orc_hemisphere_sample(n, *[_p(c) for c in wi], _p(u1), _p(u2), method,
                                  *[_p(c) for c in h])
    return np.stack(h, axis=-1)


def vndf_sample(wi, ax, ay, u1=None, u2=None, seed=0, index_base=0, method=CAP,
                nthreads=0):
    """General VNDF sampler (Sec. 2) with the cap (Sec. 3.3) or disk hemisphere
    routine; returns (h[n,3], pdf[n]) with the pdf of Eq. (1) at h."""
    wi = [_f64(c) for c in wi]
    n = wi[0].shape[0]
    ax = _f64(ax, n)
    ay = _f64(ay, n)
    if (u1 is None) != (u2 is None):
        raise ValueError("u1 and u2 must both be given or both be None")
    if u1 is not None:
        u1 = _f64(u1, n)
        u2 = _f64(u2, n)
    h = [np.zeros(n) for _ in range(3)]
    pdf = np.zeros(n)
    rc = _load().orc_vndf_sample(n, *[_p(c) for c in wi], _p(ax), _p(ay), _p(u1), _p(u2),
                                 seed, index_base, method, *[_p(c) for c in h], _p(pdf),
                                 _nt(nthreads))
    if rc != 0:
        raise ValueError("orc_vndf_sample failed")
    return np.stack(h, axis=-1), pdf


def vndf_pdf(wi, h, ax, ay, nthreads=0):
    """VNDF pdf of Eq. (1) at caller-given normals."""
    wi = [_f64(c) for c in wi]
    n = wi[0].shape[0]
    h = [_f64(c) for c in h]
    ax = _f64(ax, n)
    ay = _f64(ay, n)
    pdf = np.zeros(n)
    rc = _load().orc_vndf_pdf(n, *[_p(c) for c in wi], *[_p(c) for c in h], _p(ax), _p(ay),
                              _p(pdf), _nt(nthreads))
    if rc != 0:
        raise ValueError("orc_vndf_pdf failed")
    return pdf


def ggx_ndf(h, ax, ay):
    """GGX NDF D(h) of Appendix A."""
    h = [_f64(c) for c in h]
    n = h[0].shape[0]
    out = np.zeros(n)
    _load().orc_ggx_ndf(n, *[_p(c) for c in h], _p(_f64(ax, n)), _p(_f64(ay, n)), _p(out))
    return out


def smith_g1(h, w, ax, ay):
    """Smith G1(h, w) of Appendix A (zero at or below the horizon)."""
    h = [_f64(c) for c in h]
    w = [_f64(c) for c in w]
    n = h[0].shape[0]
    out = np.zeros(n)
    _load().orc_smith_g1(n, *[_p(c) for c in h], *[_p(c) for c in w], _p(_f64(ax, n)),
                         _p(_f64(ay, n)), _p(out))
    return out


def brdf(ax, ay, wa, wb, f0):
    """Cook-Torrance GGX BRDF f_r(wa, wb) of Appendix A with Schlick Fresnel."""
    wa = [_f64(c) for c in wa]
    wb = [_f64(c) for c in wb]
    n = wa[0].shape[0]
    out = np.zeros(n)
    _load().orc_brdf(n, _p(_f64(ax, n)), _p(_f64(ay, n)), *[_p(c) for c in wa],
                     *[_p(c) for c in wb], float(f0), _p(out))
    return out


def albedo_terms(wo, ax, ay, u1, u2, f0=1.0, method=CAP):
    """Single estimator terms f_r |cos| / PDF (Appendix A) for given uniforms."""
    wo = [_f64(c) for c in wo]
    n = wo[0].shape[0]
    out = np.zeros(n)
    _load().orc_albedo_terms(n, *[_p(c) for c in wo], _p(_f64(ax, n)), _p(_f64(ay, n)),
                             _p(_f64(u1, n)), _p(_f64(u2, n)), float(f0), method, _p(out))
    return out


def _cells(wo, ax, ay, nsamples, units, f0):
    wo = [_f64(c) for c in wo]
    n = wo[0].shape[0]
    ax = _f64(ax, n)
    ay = _f64(ay, n)
    ns = np.ascontiguousarray(np.broadcast_to(np.asarray(nsamples, dtype=np.int64), (n,)))
    un = None
    if units is not None:
        un = np.ascontiguousarray(np.asarray(units, dtype=np.uint32).reshape(n))
    f0 = _f64(f0, n)
    return wo, n, ax, ay, ns, un, f0


def albedo(wo, ax, ay, nsamples, seed, f0=1.0, units=None, method=CAP, nthreads=0):
    """Directional albedo per cell: the MC estimator of Appendix A with L == 1
    over the Philox stream (seed, tag 3, unit = units[c] or c)."""
    wo, n, ax, ay, ns, un, f0 = _cells(wo, ax, ay, nsamples, units, f0)
    out = np.zeros(n)
    rc = _load().orc_albedo(n, *[_p(c) for c in wo], _p(ax), _p(ay), ns.ctypes.data_as(_i64),
                            None if un is None else un.ctypes.data_as(_u32), seed, _p(f0),
                            method, _p(out), _nt(nthreads))
    if rc != 0:
        raise ValueError("orc_albedo failed")
    return out


def albedo_grad(wo, ax, ay, nsamples, seed, f0=1.0, units=None, nthreads=0):
    """(albedo, d/d alpha_x, d/d alpha_y, d/d theta_o) per cell by dual numbers."""
    wo, n, ax, ay, ns, un, f0 = _cells(wo, ax, ay, nsamples, units, f0)
    outs = [np.zeros(n) for _ in range(4)]
    rc = _load().orc_albedo_grad(n, *[_p(c) for c in wo], _p(ax), _p(ay),
                                 ns.ctypes.data_as(_i64),
                                 None if un is None else un.ctypes.data_as(_u32), seed,
                                 _p(f0), *[_p(c) for c in outs], _nt(nthreads))
    if rc != 0:
        raise ValueError("orc_albedo_grad failed")
    return tuple(outs)


def albedo_fd(wo, ax, ay, nsamples, seed, f0=1.0, step=1e-4, units=None, nthreads=0):
    """Central finite differences of ``albedo`` (same random numbers)."""
    wo, n, ax, ay, ns, un, f0 = _cells(wo, ax, ay, nsamples, units, f0)
    outs = [np.zeros(n) for _ in range(3)]
    rc = _load().orc_albedo_fd(n, *[_p(c) for c in wo], _p(ax), _p(ay),
                               ns.ctypes.data_as(_i64),
                               None if un is None else un.ctypes.data_as(_u32), seed,
                               _p(f0), float(step), *[_p(c) for c in outs], _nt(nthreads))
    if rc != 0:
        raise ValueError("orc_albedo_fd failed")
    return tuple(outs)


def albedo_kinks(wo, ax, ay, nsamples, seed, step=1e-4, units=None, nthreads=0):
    """Per cell, for alpha_x, alpha_y and theta_o: the number of samples whose
    estimator term is zero at some and non-zero at others of the parameter
    minus step, at it and plus step (the reflection crosses the horizon
    within the step, a kink of the term)."""
    wo, n, ax, ay, ns, un, _ = _cells(wo, ax, ay, nsamples, units, 1.0)
    outs = [np.zeros(n, dtype=np.int64) for _ in range(3)]
    rc = _load().orc_albedo_kinks(n, *[_p(c) for c in wo], _p(ax), _p(ay),
                                  ns.ctypes.data_as(_i64),
                                  None if un is None else un.ctypes.data_as(_u32), seed,
                                  float(step), *[c.ctypes.data_as(_i64) for c in outs],
                                  _nt(nthreads))
    if rc != 0:
        raise ValueError("orc_albedo_kinks failed")
    return tuple(outs)


# First-order rounding bound of the reflected direction's z in the FP32
# estimator kernels, in units of 2^-24: (HORIZON_C0 + HORIZON_C1 kappa).  The
# kernels' normal is within (8 + 48 kappa) 2^-24 of the exact one (the cap
# sampler's count); wl = 2 (wo.h) h - wo multiplies that by 4 and adds the
# roundings of the dot product, the reflection and wo's normalisation.
HORIZON_C0 = 44.0
HORIZON_C1 = 192.0


def albedo_horizon_band(wo, ax, ay, nsamples, seed, f0=1.0, c0=HORIZON_C0, c1=HORIZON_C1,
                        kappa_max=float("inf"), units=None, nthreads=0):
    """Per cell: (bound on |d/d alpha_x|, |d/d alpha_y|, |d/d theta_o| of the
    change a side flip of near-horizon samples can make, count of those
    samples).  See orc_albedo_horizon_band in oracle.cpp."""
    wo, n, ax, ay, ns, un, f0 = _cells(wo, ax, ay, nsamples, units, f0)
    outs = [np.zeros(n) for _ in range(3)]
    cnt = np.zeros(n, dtype=np.int64)
    rc = _load().orc_albedo_horizon_band(n, *[_p(c) for c in wo], _p(ax), _p(ay),
                                         ns.ctypes.data_as(_i64),
                                         None if un is None else un.ctypes.data_as(_u32),
                                         seed, _p(f0), float(c0), float(c1), float(kappa_max),
                                         *[_p(c) for c in outs], cnt.ctypes.data_as(_i64),
                                         _nt(nthreads))
    if rc != 0:
        raise ValueError("orc_albedo_horizon_band failed")
    return (*outs, cnt)


def _lobes(lobes):
    lb = np.ascontiguousarray(np.asarray(lobes, dtype=np.float64).reshape(-1, 5))
    return lb, lb.shape[0]


def radiance_at(w, lobes):
    """Synthetic radiance L(w) = sum_k lambda_k exp(kappa_k (mu_k . w - 1)) at unit w;
    lobes is an array of rows (mu_x, mu_y, mu_z, kappa, lambda)."""
    w = [_f64(c) for c in w]
    n = w[0].shape[0]
    lb, k = _lobes(lobes)
    out = np.zeros(n)
    _load().orc_radiance_at(n, *[_p(c) for c in w], _p(lb), k, _p(out))
    return out


def radiance(wo, ax, ay, nsamples, seed, lobes, f0=1.0, units=None, nthreads=0):
    """Direct illumination per cell (Appendix A estimator with the lobe
    radiance), over the Philox stream (seed, tag 3, unit = units[c] or c)."""
    wo, n, ax, ay, ns, un, f0 = _cells(wo, ax, ay, nsamples, units, f0)
    lb, k = _lobes(lobes)
    out = np.zeros(n)
    rc = _load().orc_radiance(n, *[_p(c) for c in wo], _p(ax), _p(ay), _p(f0),
                              ns.ctypes.data_as(_i64),
                              None if un is None else un.ctypes.data_as(_u32), seed, _p(lb), k,
                              _p(out), _nt(nthreads))
    if rc != 0:
        raise ValueError("orc_radiance failed")
    return out


def vndf_inverse(wi, h, ax, ay, nthreads=0):
    """Inverse of the cap sampler through the reflection law (Sec. 3.2):
    (u1, u2) with u = -1 outside the domain."""
    wi = [_f64(c) for c in wi]
    n = wi[0].shape[0]
    h = [_f64(c) for c in h]
    u1 = np.zeros(n)
    u2 = np.zeros(n)
    rc = _load().orc_vndf_inverse(n, *[_p(c) for c in wi], *[_p(c) for c in h],
                                  _p(_f64(ax, n)), _p(_f64(ay, n)), _p(u1), _p(u2),
                                  _nt(nthreads))
    if rc != 0:
        raise ValueError("orc_vndf_inverse failed")
    return u1, u2


def dielectric_sample(wi, ax, ay, eta, u=None, seed=0, index_base=0, nthreads=0):
    """Rough-dielectric sampler: a cap-sampled visible normal h (Sec. 3.3), the
    lobe from u3 against the Fresnel reflectance, then reflection or Snell
    refraction about h (Walter et al. 2007).  ``u`` is None (dielectric Philox
    stream) or (u1, u2, u3).  Returns a dict with wo[n,3], pdf, weight
    (= f |wo.n| / pdf), lobe (0 reflect, 1 transmit, -1 outside the domain)
    and h[n,3]."""
    wi = [_f64(c) for c in wi]
    n = wi[0].shape[0]
    ax = _f64(ax, n)
    ay = _f64(ay, n)
    us = [None, None, None] if u is None else [_f64(c, n) for c in u]
    wo = [np.zeros(n) for _ in range(3)]
    h = [np.zeros(n) for _ in range(3)]
    pdf = np.zeros(n)
    weight = np.zeros(n)
    lobe = np.zeros(n, dtype=np.int32)
    rc = _load().orc_dielectric_sample(
        n, *[_p(c) for c in wi], _p(ax), _p(ay), float(eta), *[_p(c) for c in us], seed,
        index_base, *[_p(c) for c in wo], _p(pdf), _p(weight),
        lobe.ctypes.data_as(_i32), *[_p(c) for c in h], _nt(nthreads))
    if rc != 0:
        raise ValueError("orc_dielectric_sample failed (eta must be > 0 and != 1)")
    return {"wo": np.stack(wo, axis=-1), "pdf": pdf, "weight": weight, "lobe": lobe,
            "h": np.stack(h, axis=-1)}


def dielectric_eval(wi, wo, ax, ay, eta, nthreads=0):
    """(pdf, bsdf) of the rough dielectric at caller-given directions
    (Walter et al. 2007, BSDF and half-vector Jacobians)."""
    wi = [_f64(c) for c in wi]
    n = wi[0].shape[0]
    wo = [_f64(c) for c in wo]
    pdf = np.zeros(n)
    bsdf = np.zeros(n)
    rc = _load().orc_dielectric_eval(n, *[_p(c) for c in wi], *[_p(c) for c in wo],
                                     _p(_f64(ax, n)), _p(_f64(ay, n)), float(eta), _p(pdf),
                                     _p(bsdf), _nt(nthreads))
    if rc != 0:
        raise ValueError("orc_dielectric_eval failed (eta must be > 0 and != 1)")
    return pdf, bsdf


def fresnel_dielectric(cos_i, eta):
    """Unpolarised Fresnel reflectance of a smooth dielectric interface."""
    c = _f64(cos_i).ravel()
    out = np.zeros(c.shape[0])
    _load().orc_fresnel_dielectric(c.shape[0], _p(c), float(eta), _p(out))
    return out


def dielectric_uniforms(n, seed, index_base=0):
    """(u1, u2, u3) of the dielectric stream for tuples index_base .. + n - 1."""
    u = [np.zeros(n) for _ in range(3)]
    _load().orc_dielectric_uniforms(n, seed, index_base, *[_p(c) for c in u])
    return tuple(u)
