"""GPU parity of the rough-dielectric sampler and its pdf (C ABI through the
Python binding) against the FP64 oracle.

Tolerance.  The GPU builds the same visible normal h as the VNDF sampler, so
h carries that path's FP32 error, O(2^-24 kappa) with kappa = 1 / |M^-T hs|
(see _gpu.py).  Reflecting or refracting wi about h multiplies it by the
derivative of wo with respect to h:
  reflection    wo = 2 c h - wi,               |dwo| <= 4 |dh|,
  transmission  wo = ((c - g) h - wi) / eta,   |dwo| <= (1 + c / g + |c - g|) |dh| / eta,
with c = wi . h and g = sqrt(eta^2 - 1 + c^2) (g -> 0 at the critical angle,
where refraction is ill-conditioned).  The pdf F p_h / (4c) or
(1 - F) p_h eta g / (c - g)^2 adds the relative sensitivities of c, F and g:
K_pdf = kappa (2 + 1 / c + |F'| / F)  or  kappa (2 + |F'| / (1 - F) + c / g^2
+ 2 (1 + c / g) / |c - g|).  The weight w = a (1 + z_i) / (z_i l_o + a), with
a = |wo_z| and l_o = |M^-1 wo|, moves by (1 + z_i) z_i (l_o + a) / (z_i l_o + a)^2
times |dwo|, plus its own rounding (K + 8).  Rule: err <= max(4e-6, C 2^-24 K) per
sample with C = 64 (wo), 128 (pdf), 64 (weight), and err <= 4e-6 on every
sample with K <= 5.  Samples whose lobe decision u3 < F lies within the FP32
error of F, or whose wo_z lies within the wo tolerance of the horizon, may
legitimately take the other branch; they are checked for validity only and
must be rare.
"""

import numpy as np
import pytest
import torch

import oracle
import workloads
from _gpu import (EPS32, N_LARGE, has_device_memory, host, kappa, large_device_tuples,
                  large_sample_indices, to_dev)

pytestmark = pytest.mark.gpu

cv = pytest.importorskip("paper_2306_05044_amd")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cv.load_library()


def _fresnel_slope(c, eta):
    h = 1e-6
    lo = np.clip(c - h, 0.0, 1.0)
    hi = np.clip(c + h, 0.0, 1.0)
    return (oracle.fresnel_dielectric(hi, eta) - oracle.fresnel_dielectric(lo, eta)) / (hi - lo)


def _conditioning(d, ref, eta, u3):
    W = np.stack([d[k].astype(np.float64) for k in ("wx", "wy", "wz")], 1)
    h = ref["h"]
    kap = kappa(h, d["wx"], d["wy"], d["wz"], d["ax"], d["ay"])
    c = np.einsum("ij,ij->i", W, h)
    g = np.sqrt(np.maximum(eta * eta - 1.0 + c * c, 0.0))
    f = oracle.fresnel_dielectric(c, eta)
    fp = np.abs(_fresnel_slope(c, eta))
    refl = ref["lobe"] == 0
    gs = np.maximum(g, 1e-30)
    a_wo = np.where(refl, 4.0, (1.0 + c / gs + np.abs(c - g)) / eta)
    k_wo = kap * a_wo
    k_pdf = np.where(refl, kap * (2.0 + 1.0 / c + fp / np.maximum(f, 1e-30)),
                     kap * (2.0 + fp / np.maximum(1.0 - f, 1e-30) + c / (gs * gs)
                            + 2.0 * (1.0 + c / gs) / np.maximum(np.abs(c - g), 1e-30)))
    ax = d["ax"].astype(np.float64)
    ay = d["ay"].astype(np.float64)
    zi = W[:, 2] / np.sqrt((ax * W[:, 0]) ** 2 + (ay * W[:, 1]) ** 2 + W[:, 2] ** 2)
    wo = ref["wo"]
    a = np.abs(wo[:, 2])
    lo = np.sqrt((ax * wo[:, 0]) ** 2 + (ay * wo[:, 1]) ** 2 + wo[:, 2] ** 2)
    # |dw/dwo| for w = a (1 + z_i) / (z_i l_o + a), a = |wo_z| (|dl_o| <= |dwo|),
    # plus the weight's own rounding (w <= 1)
    k_w = k_wo * (1.0 + zi) * zi * (lo + a) / (zi * lo + a) ** 2 + 8.0
    # lobe decision within reach of FP32 error in F
    near_lobe = np.abs(u3 - f) <= 64 * EPS32 * (1.0 + fp * kap)
    near_horizon = np.abs(ref["wo"][:, 2]) <= np.maximum(4e-6, 64 * EPS32 * k_wo)
    return k_wo, k_pdf, k_w, near_lobe | near_horizon


def _check(err, k, c, name, mask):
    lim = np.maximum(4e-6, c * EPS32 * k)
    bad = (err > lim) & mask
    assert not bad.any(), f"{name}: {bad.sum()} over the limit, worst {err[bad].max():.3e} " \
        f"(K {k[bad][np.argmax(err[bad])]:.3e})"
    well = mask & (k <= 5.0)
    if well.any():
        assert np.all(err[well] <= 4e-6), f"{name}: well-conditioned max {err[well].max():.3e}"
    r = err[mask] / (EPS32 * k[mask])
    print(f"{name}: max err {err[mask].max():.3e}, max err/(eps K) {r.max():.2f}, "
          f"fraction > 4e-6 {(err[mask] > 4e-6).mean():.2e}")


def _stream_u(seed, index_base, n=None, indices=None):
    """The oracle's uniforms at contiguous positions, or at given ones."""
    if indices is None:
        return oracle.dielectric_uniforms(n, seed, index_base)
    cols = [oracle.dielectric_uniforms(1, seed, index_base + int(k)) for k in indices]
    return tuple(np.concatenate([c[j] for c in cols]) for j in range(3))


def _compare(d, outs, eta, u, name):
    """outs: GPU (wox, woy, woz, pdf, weight) as tensors or arrays; u: the
    stream's uniforms at the same tuples."""
    wi = (d["wx"], d["wy"], d["wz"])
    ref = oracle.dielectric_sample(wi, d["ax"], d["ay"], float(np.float32(eta)), u=u)
    outs = [host(x) if torch.is_tensor(x) else x for x in outs]
    wo = np.stack([x.astype(np.float64) for x in outs[:3]], 1)
    pdf = outs[3].astype(np.float64)
    wt = outs[4].astype(np.float64)
    k_wo, k_pdf, k_w, ambiguous = _conditioning(d, ref, eta, u[2])
    assert ambiguous.sum() <= max(2, 1e-3 * len(ambiguous)), ambiguous.sum()
    ok = ~ambiguous
    both = ok & (ref["pdf"] > 0)
    assert np.array_equal(pdf[ok] > 0, ref["pdf"][ok] > 0), f"{name}: validity differs"
    _check(np.linalg.norm(wo - ref["wo"], axis=1), k_wo, 64, name + " wo", ok)
    rel = np.abs(pdf[both] / ref["pdf"][both] - 1.0)
    full = np.zeros_like(pdf)
    full[both] = rel
    _check(full, k_pdf, 128, name + " pdf", both)
    _check(np.abs(wt - ref["weight"]), k_w, 64, name + " weight", ok)
    # every GPU sample, ambiguous ones included, is a valid sample or no
    # sample: finite, a weight in [0, 1] and a unit direction, each up to the
    # same per-sample error bound as the comparisons above (wo loses up to
    # 64 2^-24 K_wo near the critical angle, and its length with it)
    assert np.all(np.isfinite(wo)) and np.all(pdf >= 0)
    w_hi = 1.0 + np.maximum(1e-6, 64 * EPS32 * k_w)
    assert np.all((wt >= 0) & (wt <= w_hi)), f"{name}: weight above 1 by {np.max(wt - w_hi):.3e}"
    gv = pdf > 0
    dn = np.abs(np.linalg.norm(wo, axis=1) - 1.0)
    n_hi = np.maximum(1e-4, 64 * EPS32 * k_wo)
    assert np.all(dn[gv] <= n_hi[gv]), f"{name}: |wo| off by {np.max(dn[gv] - n_hi[gv]):.3e}"
    return ref


@pytest.mark.parametrize("eta", [1.5, 1.0 / 1.5, 1.33, 2.4])
def test_small_config_parity(eta):
    """65,536 isotropic tuples (roughness log-uniform in [0.01, 1]), all compared."""
    d = workloads.tuples_small(65536, seed=0)
    t = to_dev(d)
    outs = cv.dielectric_sample(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], eta, seed=7)
    _compare(d, outs, eta, _stream_u(7, 0, 65536), f"eta {eta:.4f}")


@pytest.mark.parametrize("eta", [1.5, 1.0 / 1.33])
def test_anisotropic_parity(eta):
    """Streaming-workload tuples: grazing views and roughness down to 1e-3."""
    d = workloads.tuples_streaming(1 << 16, seed=12)
    t = to_dev(d)
    outs = cv.dielectric_sample(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], eta, seed=3,
                                index_base=1 << 33)
    _compare(d, outs, eta, _stream_u(3, 1 << 33, 1 << 16), f"aniso eta {eta:.4f}")


@pytest.mark.parametrize("eta", [1.0005, 1.0 / 1.0005, 4.0])
def test_extreme_indices(eta):
    """Nearly index-matched media (the refracted ray barely bends and the
    transmission pdf is sharply peaked) and a very dense one."""
    d = workloads.tuples_small(1 << 14, seed=4)
    t = to_dev(d)
    outs = cv.dielectric_sample(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], eta, seed=5)
    assert all(torch.all(torch.isfinite(o)).item() for o in outs)
    _compare(d, outs, eta, _stream_u(5, 0, 1 << 14), f"eta {eta:.5f}")


@pytest.mark.parametrize("n", [1, 3, 4, 5, 63, 65, 1023, 4097])
def test_ragged_sizes_and_scalar_path(n):
    d = workloads.tuples_streaming(n + 1, seed=21)
    t = to_dev(d)
    a = cv.dielectric_sample(t["wx"][:n], t["wy"][:n], t["wz"][:n], t["ax"][:n], t["ay"][:n],
                             1.5, seed=9, index_base=5)
    _compare({k: v[:n] for k, v in d.items()}, a, 1.5, _stream_u(9, 5, n), f"n={n}")
    # misaligned copies of the same values take the scalar path: same bits
    buf = {k: torch.zeros(n + 1, device="cuda") for k in t}
    for k in t:
        buf[k][1:].copy_(t[k][:n])
    b = cv.dielectric_sample(buf["wx"][1:], buf["wy"][1:], buf["wz"][1:], buf["ax"][1:],
                             buf["ay"][1:], 1.5, seed=9, index_base=5)
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    # a split call continues the stream: the second half at index_base + m
    m = n // 2
    if m > 0:
        c2 = cv.dielectric_sample(t["wx"][m:n], t["wy"][m:n], t["wz"][m:n], t["ax"][m:n],
                                  t["ay"][m:n], 1.5, seed=9, index_base=5 + m)
        for x, y in zip(a, c2):
            assert torch.equal(x[m:n], y)


def test_domain_edges_and_total_reflection():
    wz = torch.tensor([1.0, 0.0, -0.5, 1.0, 1.0, 0.2, 0.05, 1.0], device="cuda")
    wx = torch.sqrt(torch.clamp(1 - wz * wz, min=0.0))
    wy = torch.zeros_like(wz)
    ax = torch.tensor([0.5, 0.5, 0.5, 0.0, 0.5, 1e-3, 1e-3, 1.0], device="cuda")
    ay = torch.tensor([0.5, 0.5, 0.5, 0.5, -1.0, 1e-3, 1e-3, 1.0], device="cuda")
    wox, woy, woz, pdf, w = cv.dielectric_sample(wx, wy, wz, ax, ay, 1.0 / 1.5, seed=1)
    O = np.stack([host(wox), host(woy), host(woz)], 1)
    for i in (1, 2, 3, 4):
        assert tuple(O[i]) == (0.0, 0.0, 1.0) and host(pdf)[i] == 0 and host(w)[i] == 0
    # from the dense side at 78 and 87 degrees, past the critical angle of
    # 41.8 degrees, a nearly smooth surface reflects everything
    for i in (5, 6):
        assert O[i, 2] > 0 and host(pdf)[i] > 0
    assert np.all(np.isfinite(O)) and np.all(np.isfinite(host(pdf)))


def _check_pdf_entry(W, O, ax, ay, eta, got, name):
    """dielectric_pdf output `got` at FP32 directions W (wi) and O (wo) vs the
    oracle at the same values and the same (FP32) eta.  The entry point works
    in double, so every density is within 2e-6 relative; a zero on one side
    only is allowed where a validity test (wi.h > 0, wo.h < 0 for
    transmission) sits within 1e-12 of its threshold."""
    eta32 = float(np.float32(eta))
    ref, _ = oracle.dielectric_eval(W, O, ax, ay, eta32)
    Wm, Om = np.stack(W, 1), np.stack(O, 1)
    refl = Om[:, 2] > 0
    tv = np.where(refl[:, None], Wm + Om, -(Wm + eta32 * Om))
    hh = tv * (np.sign(tv[:, 2]) / np.linalg.norm(tv, axis=1))[:, None]
    ci = np.einsum("ij,ij->i", Wm, hh)
    co = np.einsum("ij,ij->i", Om, hh)
    edge = (np.abs(ci) < 1e-12) | (~refl & (np.abs(co) < 1e-12))
    both = (ref > 0) & (got > 0)
    one = (ref > 0) != (got > 0)
    assert not (one & ~edge).any(), (one & ~edge).sum()
    rel = np.abs(got[both] / ref[both] - 1)
    print(f"{name}: {both.sum()} densities, max rel {rel.max():.2e}")
    assert np.all(rel <= 2e-6), rel.max()


def test_pdf_entry_point():
    """dielectric_pdf at FP32 directions vs the oracle at the same values."""
    n = 65536 + 3
    d = workloads.tuples_streaming(n, seed=8)
    t = to_dev(d)
    for eta in (1.5, 1.0 / 1.5):
        wox, woy, woz, _, _ = cv.dielectric_sample(t["wx"], t["wy"], t["wz"], t["ax"],
                                                       t["ay"], eta, seed=2)
        p = cv.dielectric_pdf(t["wx"], t["wy"], t["wz"], wox, woy, woz, t["ax"], t["ay"], eta)
        O = [host(x).astype(np.float64) for x in (wox, woy, woz)]
        W = [d[k].astype(np.float64) for k in ("wx", "wy", "wz")]
        _check_pdf_entry(W, O, d["ax"], d["ay"], eta, host(p).astype(np.float64),
                         f"pdf entry eta {eta:.4f}")


def test_explicit_uniforms_match_the_stream():
    """Caller-given (u1, u2, u3) equal to the stream's give the same bits, on
    the vector path and (through misaligned copies) the scalar path."""
    n = 4099
    d = workloads.tuples_small(n, seed=3)
    t = to_dev(d)
    a = cv.dielectric_sample(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], 1.5, seed=11,
                             index_base=7)
    u = [torch.from_numpy(x.astype(np.float32)).cuda() for x in oracle.dielectric_uniforms(n, 11, 7)]
    b = cv.dielectric_sample(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], 1.5, u=u)
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    bufs = []
    for x in u:
        buf = torch.zeros(n + 1, device="cuda")
        buf[1:].copy_(x)
        bufs.append(buf[1:])
    c = cv.dielectric_sample(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], 1.5, u=bufs)
    for x, y in zip(a, c):
        assert torch.equal(x, y)


def test_determinism():
    d = workloads.tuples_streaming(1 << 16, seed=1)
    t = to_dev(d)
    a = cv.dielectric_sample(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], 1.5, seed=1)
    b = cv.dielectric_sample(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], 1.5, seed=1)
    for x, y in zip(a, b):
        assert torch.equal(x, y)


@pytest.mark.parametrize("eta", [1.5, 1.0 / 1.5])
def test_streaming_full_size_every_sample(eta):
    """All 2^26 anisotropic tuples in the benchmark's launch configuration
    against the oracle on every sample (rules as above), and the invariants
    on all of them."""
    n = 1 << 26
    d = workloads.tuples_streaming(n, seed=1)
    t = to_dev(d)
    outs = cv.dielectric_sample(t["wx"], t["wy"], t["wz"], t["ax"], t["ay"], eta, seed=1)
    torch.cuda.synchronize()
    del t
    wox, woy, woz, pdf, w = outs
    assert torch.all(torch.isfinite(pdf)) and torch.all(pdf >= 0)
    valid = pdf > 0
    assert valid.double().mean().item() > (0.97 if eta > 1 else 0.5)
    got = [host(x) for x in outs]
    del outs, wox, woy, woz, pdf, w, valid
    _compare(d, got, eta, _stream_u(1, 0, n=n), f"2^26 every sample eta {eta:.4f}")


def test_more_than_one_launch_sampled():
    """n = 2^31 + 3 * 2^20 + 5 tuples resident in HBM (eta = 1.5): the sampler
    (vector and scalar paths) and the pdf entry point run as two launches;
    outputs at the start, on both sides of the 2^31 boundary, at the ragged
    tail and at 2048 random positions against the oracle at the same stream
    positions."""
    if not has_device_memory(160):
        pytest.skip("needs about 90 GB of device memory")
    n = N_LARGE
    idx = large_sample_indices(n, 2048, seed=4)
    it = torch.from_numpy(idx).cuda()
    t = large_device_tuples(n, seed=22)
    u = _stream_u(12, 0, indices=idx)
    try:
        for off in (0, 1):  # aligned arrays (vector path), then offset views (scalar path)
            v = {k: x[off:off + n] for k, x in t.items()}
            outs = cv.dielectric_sample(v["wx"], v["wy"], v["wz"], v["ax"], v["ay"], 1.5, seed=12)
            torch.cuda.synchronize()
            sub = {k: host(x[it]) for k, x in v.items()}
            _compare(sub, [x[it] for x in outs], 1.5, u, f"2^31+ offset {off}")
            if off == 0:
                wox, woy, woz = outs[:3]
                q = cv.dielectric_pdf(v["wx"], v["wy"], v["wz"], wox, woy, woz, v["ax"], v["ay"],
                                      1.5)
                torch.cuda.synchronize()
                O = [host(x[it]).astype(np.float64) for x in (wox, woy, woz)]
                W = [sub[k].astype(np.float64) for k in ("wx", "wy", "wz")]
                _check_pdf_entry(W, O, sub["ax"], sub["ay"], 1.5, host(q[it]).astype(np.float64),
                                 "pdf entry 2^31+")
                del wox, woy, woz, q
            del outs, v
    finally:
        del t
        torch.cuda.empty_cache()
