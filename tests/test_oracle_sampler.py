"""Pins of the oracle's VNDF samplers (CPU only).

What fixes each part of the sampler without another implementation of it:

* invariants of the construction (unit h above the horizon, facing wi);
* the exact inverse map through the reflection law and the half vector
  (Sec. 3.2): from h, wi and alpha the cap point c and then (u1, u2) are
  recovered, which pins the azimuth/height roles and the cap bounds;
* normal incidence, where the VNDF is D(h) h_z and the textbook inversion of
  the GGX NDF (Walter et al. 2007) gives h in closed form, anisotropic too
  (this pins which of alpha_x / alpha_y stretches which axis);
* the uniform density of the cap, 1 / (2 pi (1 + z_i)) (Sec. 3.2);
* a chi-square test of the samples against the pdf of Eq. (1) integrated per
  bin, and a two-sample test of the cap sampler against Heitz's disk sampler.
"""

import numpy as np
import pytest
from scipy import stats

from _hemi import binned_grid, slope_coords
import workloads


def _wi(mu, phi, n):
    s = np.sqrt(1.0 - mu * mu)
    return (np.full(n, s * np.cos(phi)), np.full(n, s * np.sin(phi)), np.full(n, mu))


CASES = [  # (ax, ay, mu, phi)
    (0.3, 0.6, 0.2, 0.7),
    (0.05, 0.05, 0.05, 0.0),
    (1.0, 1.0, 0.9, 2.0),
    (0.01, 0.2, 0.5, 4.0),
    (0.8, 0.02, 0.7, 5.5),
]


@pytest.mark.parametrize("method", [0, 1])
def test_invariants(orc, method):
    d = workloads.tuples_small(20000, seed=11)
    wi = (d["wx"], d["wy"], d["wz"])
    h, pdf = orc.vndf_sample(wi, d["ax"], d["ay"], seed=5, method=method)
    assert np.allclose(np.linalg.norm(h, axis=1), 1.0, atol=1e-14)
    assert np.all(h[:, 2] > 0.0)
    w = np.stack([c.astype(np.float64) for c in wi], axis=1)
    assert np.all(np.einsum("ij,ij->i", h, w) >= 0.0)
    assert np.all(pdf > 0.0) and np.all(np.isfinite(pdf))


def test_inverse_map_recovers_uniforms(orc):
    """Reflect -ws about the standard-space normal to get the cap point c, then
    read u2 from its height and u1 from its azimuth."""
    d = workloads.tuples_streaming(20000, seed=12)
    wi = np.stack([d["wx"], d["wy"], d["wz"]], axis=1).astype(np.float64)
    ax = d["ax"].astype(np.float64)
    ay = d["ay"].astype(np.float64)
    u1, u2 = orc.uniforms(3, orc.TAG_SAMPLE, 0, 0, len(ax))
    h, _ = orc.vndf_sample(tuple(wi.T), ax, ay, u1=u1, u2=u2, method=0)
    hs = np.stack([h[:, 0] / ax, h[:, 1] / ay, h[:, 2]], axis=1)
    hs /= np.linalg.norm(hs, axis=1, keepdims=True)
    ws = np.stack([wi[:, 0] * ax, wi[:, 1] * ay, wi[:, 2]], axis=1)
    ws /= np.linalg.norm(ws, axis=1, keepdims=True)
    c = 2.0 * np.einsum("ij,ij->i", hs, ws)[:, None] * hs - ws
    zs = ws[:, 2]
    u2_rec = 1.0 - (c[:, 2] + zs) / (1.0 + zs)
    u1_rec = np.mod(np.arctan2(c[:, 1], c[:, 0]) / (2 * np.pi), 1.0)
    # the map is well conditioned away from the cap's apex and poles of c
    ok = np.hypot(c[:, 0], c[:, 1]) > 1e-3
    assert np.max(np.abs(u2_rec - u2)) < 1e-9
    du1 = np.abs(u1_rec - u1)
    du1 = np.minimum(du1, 1.0 - du1)
    assert np.max(du1[ok]) < 1e-9
    # |c| = 1: the reflected direction lies on the unit sphere, inside the cap
    assert np.allclose(np.linalg.norm(c, axis=1), 1.0, atol=1e-12)
    assert np.all(c[:, 2] > -zs - 1e-12)


@pytest.mark.parametrize("ax,ay", [(0.3, 0.3), (0.05, 0.7), (1.0, 0.01)])
def test_normal_incidence_textbook_inversion(orc, ax, ay):
    """At wi = e_z the VNDF is D(h) h_z, whose inverse-CDF sample is
    h ~ (ax sqrt(u2) cos 2 pi u1, ay sqrt(u2) sin 2 pi u1, sqrt(1 - u2))."""
    n = 5000
    u1, u2 = orc.uniforms(21, orc.TAG_SAMPLE, 0, 0, n)
    wi = (np.zeros(n), np.zeros(n), np.ones(n))
    ref = np.stack([ax * np.sqrt(u2) * np.cos(2 * np.pi * u1),
                    ay * np.sqrt(u2) * np.sin(2 * np.pi * u1), np.sqrt(1.0 - u2)], axis=1)
    ref /= np.linalg.norm(ref, axis=1, keepdims=True)
    for method in (0, 1):
        h, _ = orc.vndf_sample(wi, np.full(n, ax), np.full(n, ay), u1=u1, u2=u2,
                               method=method)
        assert np.max(np.abs(h - ref)) < 1e-12
    if ax == ay:
        # isotropic: tan^2(theta_h) = alpha^2 u2 / (1 - u2), phi_h = 2 pi u1
        h, _ = orc.vndf_sample(wi, np.full(n, ax), np.full(n, ay), u1=u1, u2=u2)
        tan2 = (h[:, 0] ** 2 + h[:, 1] ** 2) / h[:, 2] ** 2
        assert np.allclose(tan2, ax * ax * u2 / (1.0 - u2), rtol=1e-10, atol=1e-300)


def test_alpha_axes(orc):
    """A tiny alpha_x keeps normals in the x = 0 plane; a tiny alpha_y in y = 0."""
    n = 4000
    wi = _wi(0.6, 0.8, n)
    h, _ = orc.vndf_sample(wi, np.full(n, 1e-4), np.full(n, 0.8), seed=1)
    assert np.max(np.abs(h[:, 0])) < 2e-3 and np.max(np.abs(h[:, 1])) > 0.3
    h, _ = orc.vndf_sample(wi, np.full(n, 0.8), np.full(n, 1e-4), seed=1)
    assert np.max(np.abs(h[:, 1])) < 2e-3 and np.max(np.abs(h[:, 0])) > 0.3


@pytest.mark.parametrize("mu", [0.05, 0.5, 1.0])
def test_cap_is_uniform(orc, mu):
    """The cap point c = (hemisphere sample) - wi is uniform on the part of the
    unit sphere above z = -z_i: height uniform on (-z_i, 1], azimuth uniform,
    independent (density 1 / (2 pi (1 + z_i)))."""
    n = 40000
    u1, u2 = orc.uniforms(31, orc.TAG_SAMPLE, 0, 0, n)
    wi = _wi(mu, 1.1, n)
    hs = orc.hemisphere_sample(wi, u1, u2, method=0)
    c = hs - np.stack(wi, axis=1)
    assert np.allclose(np.linalg.norm(c, axis=1), 1.0, atol=1e-12)
    zc = (c[:, 2] + mu) / (1.0 + mu)
    assert stats.kstest(zc, "uniform").pvalue > 1e-3
    az = np.mod(np.arctan2(c[:, 1], c[:, 0]) / (2 * np.pi), 1.0)
    assert stats.kstest(az, "uniform").pvalue > 1e-3
    # height and azimuth independent: 2-D histogram is flat
    hist, _, _ = np.histogram2d(zc, az, bins=8, range=[[0, 1], [0, 1]])
    assert stats.chisquare(hist.ravel()).pvalue > 1e-3


def _bin_probabilities(orc, ax, ay, wi1, b_edges, p_edges):
    """Expected probability of each (beta, phi) bin: Gauss-Legendre quadrature
    of the pdf of Eq. (1) inside every bin."""
    h, w, idx = binned_grid(ax, ay, b_edges, p_edges, nq=16)
    n = h.shape[0]
    pdf = orc.vndf_pdf(tuple(np.full(n, c) for c in wi1), (h[:, 0], h[:, 1], h[:, 2]),
                       np.full(n, ax), np.full(n, ay))
    nbins = (len(b_edges) - 1) * (len(p_edges) - 1)
    return np.bincount(idx, weights=pdf * w, minlength=nbins).reshape(
        len(b_edges) - 1, len(p_edges) - 1)


def _hist(h, ax, ay, b_edges, p_edges):
    beta, phi = slope_coords(h, ax, ay)
    H, _, _ = np.histogram2d(beta, phi, bins=[b_edges, p_edges])
    return H


@pytest.mark.parametrize("ax,ay,mu,phi", CASES)
def test_chi2_against_pdf(orc, ax, ay, mu, phi):
    n = 200000
    s = np.sqrt(1 - mu * mu)
    wi1 = (s * np.cos(phi), s * np.sin(phi), mu)
    b_edges = np.linspace(0, np.pi / 2, 17)
    p_edges = np.linspace(0, 2 * np.pi, 33)
    probs = _bin_probabilities(orc, ax, ay, wi1, b_edges, p_edges)
    assert abs(probs.sum() - 1.0) < 1e-6
    for method in (0, 1):
        h, _ = orc.vndf_sample(_wi(mu, phi, n), np.full(n, ax), np.full(n, ay), seed=77,
                               method=method)
        H = _hist(h, ax, ay, b_edges, p_edges)
        exp = probs.ravel() * n
        obs = H.ravel()
        keep = exp >= 5.0
        # no samples where the pdf has (numerically) no mass
        assert obs[exp < 1e-6].sum() == 0
        o = np.append(obs[keep], obs[~keep].sum())
        e = np.append(exp[keep], exp[~keep].sum())
        if e[-1] < 5.0:
            o, e = o[:-1], e[:-1]
        e = e * o.sum() / e.sum()
        p = stats.chisquare(o, e).pvalue
        assert p > 1e-4, (method, p)


@pytest.mark.parametrize("ax,ay,mu,phi", CASES[:3])
def test_cap_matches_disk_two_sample(orc, ax, ay, mu, phi):
    n = 200000
    b_edges = np.linspace(0, np.pi / 2, 17)
    p_edges = np.linspace(0, 2 * np.pi, 33)
    hc, _ = orc.vndf_sample(_wi(mu, phi, n), np.full(n, ax), np.full(n, ay), seed=101,
                            method=0)
    hd, _ = orc.vndf_sample(_wi(mu, phi, n), np.full(n, ax), np.full(n, ay), seed=202,
                            method=1)
    A = _hist(hc, ax, ay, b_edges, p_edges).ravel()
    B = _hist(hd, ax, ay, b_edges, p_edges).ravel()
    keep = (A + B) >= 10
    table = np.stack([A[keep], B[keep]])
    p = stats.chi2_contingency(table)[1]
    assert p > 1e-4


def test_domain_and_stream_offset(orc):
    n = 6
    wi = (np.zeros(n), np.zeros(n), np.array([1.0, 0.0, -0.5, 1.0, 1.0, 0.5]))
    ax = np.array([0.5, 0.5, 0.5, 0.0, 0.5, -1.0])
    ay = np.array([0.5, 0.5, 0.5, 0.5, 0.0, 0.5])
    h, pdf = orc.vndf_sample(wi, ax, ay, seed=1)
    assert pdf[0] > 0.0
    for i in range(1, 6):
        assert tuple(h[i]) == (0.0, 0.0, 1.0) and pdf[i] == 0.0
    d = workloads.tuples_small(300, seed=2)
    wi = (d["wx"], d["wy"], d["wz"])
    hA, pA = orc.vndf_sample(wi, d["ax"], d["ay"], seed=4, index_base=0)
    hB, pB = orc.vndf_sample(tuple(c[100:] for c in wi), d["ax"][100:], d["ay"][100:],
                             seed=4, index_base=100)
    assert np.array_equal(hA[100:], hB) and np.array_equal(pA[100:], pB)


def test_oracle_inverse_map_round_trip(orc):
    """The oracle's inverse (reflection law of Sec. 3.2) undoes its cap sampler,
    and marks inputs outside the domain with -1."""
    d = workloads.tuples_streaming(20000, seed=14)
    wi = tuple(d[k].astype(np.float64) for k in ("wx", "wy", "wz"))
    u1, u2 = orc.uniforms(7, orc.TAG_SAMPLE, 0, 0, 20000)
    h, _ = orc.vndf_sample(wi, d["ax"], d["ay"], u1=u1, u2=u2, method=0)
    r1, r2 = orc.vndf_inverse(wi, tuple(h.T), d["ax"], d["ay"])
    assert np.max(np.abs(r2 - u2)) < 1e-9
    du1 = np.abs(r1 - u1)
    du1 = np.minimum(du1, 1.0 - du1)
    # the azimuth is undefined at the apex of the cap (u2 = 0) and ill-posed near it
    ok = u2 > 1e-6
    assert np.max(du1[ok]) < 1e-7
    assert np.all((r1 >= 0) & (r1 < 1) & (r2 >= -1e-12) & (r2 < 1 + 1e-12))
    n = 4
    bad1, bad2 = orc.vndf_inverse((np.zeros(n), np.zeros(n), np.array([-1.0, 1.0, 1.0, 1.0])),
                                  (np.zeros(n), np.array([0.0, 0.0, 1.0, 0.0]),
                                   np.array([1.0, -0.5, 0.0, 1.0])),
                                  np.array([0.5, 0.5, 0.5, 0.0]), np.full(n, 0.5))
    assert np.all(bad1 == -1.0) and np.all(bad2 == -1.0)


def _degenerate_tuples():
    """Rim (u2 = 1 - 2^-24) and apex of the cap, quadrant azimuths, normal
    incidence, near-grazing views, extreme roughness: the GPU tests' set."""
    u2s = [0.0, 2.0 ** -24, 0.5, 1.0 - 2.0 ** -24]
    u1s = [0.0, 0.25, 0.5, 0.75, 1.0 - 2.0 ** -24]
    views = [(0.0, 0.0, 1.0), (np.sqrt(1 - 1e-6), 0.0, 1e-3), (0.6, 0.0, 0.8),
             (0.0, -np.sqrt(1 - 1e-8), 1e-4)]
    alphas = [(1.0, 1.0), (1e-3, 1e-3), (1e-5, 0.5), (0.5, 1e-5), (1.0, 1e-3)]
    rows = [(v, a, p, q) for v in views for a in alphas for p in u1s for q in u2s]
    f = np.float32
    w = tuple(np.array([r[0][i] for r in rows], f).astype(np.float64) for i in range(3))
    ax = np.array([r[1][0] for r in rows], f).astype(np.float64)
    ay = np.array([r[1][1] for r in rows], f).astype(np.float64)
    u1 = np.array([r[2] for r in rows], f).astype(np.float64)
    u2 = np.array([r[3] for r in rows], f).astype(np.float64)
    return w, ax, ay, u1, u2


def test_ill_conditioned_samples(orc):
    """Samples at the rim of the cap opposite to the view, where the half
    vector is the sum of two nearly opposite unit vectors (conditioning up to
    about 2^24): the oracle's pdf, evaluated through Eq. (1), equals the fused
    form L^3 / (pi ax ay (1 + zs) |hs|^2) of the same density (an identity of
    Appendix A's quantities, evaluated here with 50 significant digits at
    the oracle's normal) within 1e-8, and the inverse map (Sec. 3.2, also at
    50 digits) takes the oracle's normal back to its u2 within 1e-9 and to
    u1 within 1e-8 turns where the cap point is off the axis.  In plain
    double precision the literal half vector loses up to 6 % of this pdf."""
    import mpmath as mp
    mp.mp.dps = 50
    w, ax, ay, u1, u2 = _degenerate_tuples()
    h, p = orc.vndf_sample(w, ax, ay, u1=u1, u2=u2)
    worst_p = worst_u2 = worst_u1 = 0.0
    for i in range(len(u1)):
        a, b = mp.mpf(ax[i]), mp.mpf(ay[i])
        wx, wy, wz = (mp.mpf(x[i]) for x in w)
        l = mp.sqrt((a * wx) ** 2 + (b * wy) ** 2 + wz ** 2)
        ws = (a * wx / l, b * wy / l, wz / l)
        hx, hy, hz = (mp.mpf(h[i, j]) for j in range(3))
        mt = (hx / a, hy / b, hz)
        n = mp.sqrt(sum(x * x for x in mt))
        hstd = tuple(x / n for x in mt)
        d = sum(x * y for x, y in zip(hstd, ws))
        hs_len = 2 * d                      # |hs| = 2 ws . h_std (|c| = |ws| = 1)
        L = hs_len / n                       # |M^-T hs| with hs = |hs| h_std
        fused = L ** 3 / (mp.pi * a * b * (1 + ws[2]) * hs_len ** 2)
        worst_p = max(worst_p, abs(float(mp.mpf(p[i]) / fused - 1)))
        c = tuple(2 * d * x - y for x, y in zip(hstd, ws))  # reflect ws about h_std
        r2 = 1 - (c[2] + ws[2]) / (1 + ws[2])
        worst_u2 = max(worst_u2, abs(float(r2) - u2[i]))
        if mp.sqrt(c[0] ** 2 + c[1] ** 2) > 1e-6:
            t = float(mp.atan2(c[1], c[0]) / (2 * mp.pi)) % 1.0
            dt = abs(t - u1[i])
            worst_u1 = max(worst_u1, min(dt, 1.0 - dt))
    print(f"ill-conditioned: pdf {worst_p:.2e}, u2 {worst_u2:.2e}, u1 {worst_u1:.2e}")
    assert worst_p <= 1e-8 and worst_u2 <= 1e-9 and worst_u1 <= 1e-8
