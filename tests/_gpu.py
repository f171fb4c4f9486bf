"""Helpers shared by the GPU parity tests: device transfer, the oracle's
stored values for the estimator workloads, and the tolerance rules the
comparisons use.

Normals and pdfs (GPU vs FP64 oracle on the same FP32 inputs and uniforms):

* The double-precision method (CAPVNDF_CAP_F64, the default and the
  benchmark's) is held to the flat bound of the target: every h within 2e-6
  (|h - h_ref|) and every pdf within 2e-6 relative.

* The FP32-arithmetic method (CAPVNDF_CAP) forms the half vector
  hs = c + ws from two unit vectors whose components carry absolute rounding
  errors, so its error grows with the conditioning
  kappa = max(1, ax, ay) / L, L = |M^-T hs| (M^-T = diag(ax, ay, 1)).  A
  first-order worst-case count of its roundings (u = 2^-24 per correctly
  rounded operation, 2u for the hardware rsq / rcp / sqrt, 2.1u absolute for
  the turn-based sin / cos, measured exhaustively over the 2^-24 lattice)
  bounds the absolute error of hs by 40u, so |h - h_ref| <= (8 + 40 kappa) u
  (direction through the unstretch, plus the normalisation's roundings), and
  the pdf L^3 / (pi ax ay (1 + zs) |hs|^2), which moves by 3 times the
  relative error of L and 2 times that of |hs| (each at most 40 kappa u),
  by (35 + 200 kappa) u.  The tests allow 20 % over these first-order counts
  for the neglected higher-order terms: (8 + 48 kappa) u and
  (40 + 240 kappa) u.  kappa is computed from the oracle's normal: with
  h_std = M^T h / |M^T h|, |hs| = 2 ws . h_std and L = |hs| / |M^T h|.  The
  fraction of samples above 2e-6 is reported.

* Heitz's disk sampler (the timing baseline) builds the hemisphere normal from
  its height above the disk, ti = sqrt(1 - t1^2 - t2^2) = ws . h_std, whose
  argument cancels at the rim: ti carries a relative error of O(2^-24 / ti^2),
  which its pdf inherits.  Its pdf is checked against 128 u (1 / L + 1 / ti^2).
"""

import importlib.util
import os

import numpy as np
import torch

EPS32 = 2.0 ** -24
# first-order worst-case bounds of the FP32-arithmetic cap sampler, in units
# of 2^-24: |h - h_ref| <= H_A + H_B kappa, pdf relative <= P_A + P_B kappa
H_A, H_B = 8.0, 48.0
P_A, P_B = 40.0, 240.0

_GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
_golden_cache = {}


def golden(part):
    """The oracle's stored values for every unit of one estimator workload
    ("lut", "grad", "batch" or "radiance"), written by
    tests/golden/make_estimator_golden.py.
    The digest of the inputs it was computed on must match the inputs the
    workload generator gives now."""
    if "mk" not in _golden_cache:
        spec = importlib.util.spec_from_file_location(
            "make_estimator_golden", os.path.join(_GOLDEN_DIR, "make_estimator_golden.py"))
        mk = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mk)
        with np.load(mk.OUT, allow_pickle=False) as f:
            _golden_cache["data"] = {k: f[k] for k in f.files}
        _golden_cache["mk"] = mk
    mk, data = _golden_cache["mk"], _golden_cache["data"]
    inputs = {"lut": mk.lut_inputs, "grad": mk.grad_inputs, "batch": mk.batch_inputs,
              "radiance": mk.radiance_inputs}[part]()
    assert str(data[f"{part}_digest"]) == mk.digest(inputs), \
        f"{part}: the stored oracle values were computed on other inputs; rerun the script"
    return data


def to_dev(arrs, dev="cuda"):
    return {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in arrs.items()}


def host(t):
    return t.detach().cpu().numpy()


def kappa(h_ref, wx, wy, wz, ax, ay):
    """1 / |M^-T hs| of the cap construction at the oracle's normal."""
    ax = np.asarray(ax, dtype=np.float64)
    ay = np.asarray(ay, dtype=np.float64)
    mt = np.stack([h_ref[:, 0] / ax, h_ref[:, 1] / ay, h_ref[:, 2]], axis=1)
    mtn = np.linalg.norm(mt, axis=1)
    hstd = mt / mtn[:, None]
    ws = np.stack([np.asarray(wx, np.float64) * ax, np.asarray(wy, np.float64) * ay,
                   np.asarray(wz, np.float64)], axis=1)
    ws /= np.linalg.norm(ws, axis=1, keepdims=True)
    hs_norm = 2.0 * np.einsum("ij,ij->i", hstd, ws)
    # the unstretch M^-T = diag(ax, ay, 1) scales hs's absolute error by up to
    # max(ax, ay, 1) before the division by L (1 inside the workloads' range)
    return np.maximum(1.0, np.maximum(ax, ay)) * mtn / hs_norm


def kappa_disk_pdf(h_ref, wx, wy, wz, ax, ay):
    """1 / L + 1 / ti^2 for the disk sampler's pdf (ti = |hs| / 2)."""
    k = kappa(h_ref, wx, wy, wz, ax, ay)
    ax = np.asarray(ax, dtype=np.float64)
    ay = np.asarray(ay, dtype=np.float64)
    mt = np.stack([h_ref[:, 0] / ax, h_ref[:, 1] / ay, h_ref[:, 2]], axis=1)
    hstd = mt / np.linalg.norm(mt, axis=1, keepdims=True)
    ws = np.stack([np.asarray(wx, np.float64) * ax, np.asarray(wy, np.float64) * ay,
                   np.asarray(wz, np.float64)], axis=1)
    ws /= np.linalg.norm(ws, axis=1, keepdims=True)
    ti = np.einsum("ij,ij->i", hstd, ws)
    return k + 1.0 / (ti * ti)


def check_conditioned(err, kap, a, b, name):
    """Every sample within (a + b kappa) 2^-24; reports the largest
    err / (2^-24 kappa) and the fraction of samples above 2e-6."""
    lim = (a + b * kap) * EPS32
    bad = err > lim
    assert not bad.any(), f"{name}: {bad.sum()} samples over the limit, worst " \
        f"{err[bad].max():.3e} at kappa {kap[bad][np.argmax(err[bad])]:.3e}"
    ratio = err / (EPS32 * kap)
    print(f"{name}: max err {err.max():.3e}, max err/(eps kappa) {ratio.max():.2f}, "
          f"max err/limit {(err / lim).max():.3f}, fraction > 2e-6 {(err > 2e-6).mean():.2e}, "
          f"max kappa {kap.max():.3e}")
    return float((err > 2e-6).mean())


def check_flat(H, P, h_ref, p_ref, name, lim=2e-6):
    """Every h within lim of the oracle's and every pdf within lim relative;
    zero pdfs exactly where the oracle's are zero."""
    herr = np.linalg.norm(H - h_ref, axis=1)
    ok = p_ref > 0
    perr = np.abs(P[ok] / p_ref[ok] - 1.0)
    print(f"{name}: max |h - h_ref| {herr.max():.2e}, max pdf rel {perr.max():.2e} "
          f"over {len(herr)} samples")
    assert herr.max() <= lim, (name, herr.max())
    assert perr.max() <= lim, (name, perr.max())
    assert np.array_equal(P > 0, ok)


# A call of more than 2^31 elements (the element-wise entry points split it
# into launches of 2^31) with a ragged tail.
N_LARGE = (1 << 31) + 3 * (1 << 20) + 5


def large_device_tuples(n, seed, pad=4):
    """The streaming workload's distribution (cos theta uniform in [1e-3, 1],
    azimuth uniform, alpha_x, alpha_y = 10^(-3U)) drawn directly on the GPU
    from a seeded torch generator, for sizes whose host copies would not fit;
    arrays hold n + pad elements so that offset views stay in bounds."""
    import math
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    t = {k: torch.empty(n + pad, device="cuda") for k in ("wx", "wy", "wz", "ax", "ay")}
    step = 1 << 27
    for o in range(0, n + pad, step):
        m = min(step, n + pad - o)

        def r():
            return torch.rand(m, generator=g, device="cuda", dtype=torch.float64)
        mu = 1e-3 + (1.0 - 1e-3) * (1.0 - r())
        phi = 2.0 * math.pi * r()
        s = torch.sqrt(1.0 - mu * mu)
        t["wx"][o:o + m] = (s * torch.cos(phi)).float()
        t["wy"][o:o + m] = (s * torch.sin(phi)).float()
        t["wz"][o:o + m] = mu.float()
        t["ax"][o:o + m] = torch.pow(10.0, -3.0 * r()).float()
        t["ay"][o:o + m] = torch.pow(10.0, -3.0 * r()).float()
    return t


def large_sample_indices(n, count, seed):
    """Sorted positions: the first elements, both sides of every 2^31 slice
    boundary, the ragged tail, and `count` random ones."""
    rng = np.random.default_rng(seed)
    fixed = [np.arange(0, 40)]
    for b in range(1 << 31, n, 1 << 31):
        fixed.append(np.arange(b - 40, b + 40))
    fixed.append(np.arange(n - 40, n))
    idx = np.concatenate(fixed + [rng.choice(n, count, replace=False)])
    return np.unique(idx)


def has_device_memory(gib):
    return torch.cuda.get_device_properties(0).total_memory >= gib * 2 ** 30
