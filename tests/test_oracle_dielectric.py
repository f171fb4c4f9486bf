"""Pins of the oracle's rough-dielectric sampler and densities (CPU only).

The paper applies its sampler to rough dielectrics and refers to Walter et
al. 2007 for the transmission model.  What fixes the oracle here is physics
and mathematics the oracle does not use in that form:

* Fresnel reflectance: normal incidence ((eta - 1) / (eta + 1))^2, zero
  p-reflectance at Brewster's angle (tan theta_B = eta), total internal
  reflection beyond the critical angle, reciprocity F(cos_i, eta) =
  F(cos_t, 1 / eta), and the amplitude form R = (r_s^2 + r_p^2) / 2 built
  from sines and cosines of the two angles;
* geometry of every sample: unit directions, the law of reflection, Snell's
  law about the sampled normal (eta |wo x h| = |wi x h|), coplanarity, and the
  half-vector reconstruction from (wi, wo);
* the smooth limit (alpha -> 0): reflection with probability F(mu) and the
  Snell direction about the macro-normal;
* normalisation: the evaluated pdf integrated over each hemisphere of
  outgoing directions (a direct quadrature over the sphere, which does not go
  through the half-vector Jacobian) equals the probability that the sampler
  produces a valid sample of that lobe;
* a chi-square test of the sampled directions against the evaluated pdf;
* the weight f |wo.n| / pdf equals the closed form (1 + L_i) / (1 + L_i + L_o)
  with Smith's Lambda;
* generalised reciprocity of the BTDF, f(wi, wo; eta) = eta^2 f(wo', wi'; 1/eta)
  in the vertically flipped frame, and symmetry of the BRDF;
* the uniforms are words 0..2 of one Philox block per sample.
"""

import math

import numpy as np
import pytest

ETAS = [1.5, 1.0 / 1.5, 1.33, 2.4]


def _unit(mu, phi, n=1):
    s = math.sqrt(max(0.0, 1.0 - mu * mu))
    return (np.full(n, s * math.cos(phi)), np.full(n, s * math.sin(phi)), np.full(n, mu))


def _lam(w, ax, ay):
    return 0.5 * (-1.0 + np.sqrt(1.0 + ((ax * w[:, 0]) ** 2 + (ay * w[:, 1]) ** 2) / w[:, 2] ** 2))


# ---------------------------------------------------------------------------
# Fresnel
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("eta", ETAS)
def test_fresnel_closed_forms(orc, eta):
    assert orc.fresnel_dielectric([1.0], eta)[0] == pytest.approx(((eta - 1) / (eta + 1)) ** 2, rel=1e-13)
    # Brewster: tan(theta_B) = eta, r_p = 0, r_s = (1 - eta^2) / (1 + eta^2)
    tb = math.atan(eta)
    rs = (1 - eta * eta) / (1 + eta * eta)
    assert orc.fresnel_dielectric([math.cos(tb)], eta)[0] == pytest.approx(rs * rs / 2, rel=1e-12)
    # grazing incidence reflects everything
    assert orc.fresnel_dielectric([0.0], eta)[0] == pytest.approx(1.0, abs=1e-15)


@pytest.mark.parametrize("eta", ETAS)
def test_fresnel_angle_form_and_reciprocity(orc, eta):
    # Fresnel's sine/tangent form: R_s = sin^2(ti - tt) / sin^2(ti + tt),
    # R_p = tan^2(ti - tt) / tan^2(ti + tt), tt from Snell's law.
    ti = np.linspace(0.01, 1.55, 200)
    st = np.sin(ti) / eta
    ok = st < 1.0
    tt = np.arcsin(np.where(ok, st, 0.0))
    rs = np.sin(ti - tt) ** 2 / np.sin(ti + tt) ** 2
    rp = np.tan(ti - tt) ** 2 / np.tan(ti + tt) ** 2
    want = np.where(ok, 0.5 * (rs + rp), 1.0)
    got = orc.fresnel_dielectric(np.cos(ti), eta)
    np.testing.assert_allclose(got, want, rtol=1e-10, atol=1e-14)
    # reciprocity: the same interface seen from the other side
    back = orc.fresnel_dielectric(np.cos(tt[ok]), 1.0 / eta)
    np.testing.assert_allclose(got[ok], back, rtol=1e-11, atol=1e-14)
    if eta < 1.0:
        crit = math.asin(eta)
        assert np.all(got[ti > crit + 1e-9] == 1.0)
        assert np.all(got[ti < crit - 1e-9] < 1.0)


# ---------------------------------------------------------------------------
# Sample geometry
# ---------------------------------------------------------------------------

GEOM = [(0.3, 0.3, 0.6, 0.4, 1.5), (0.05, 0.5, 0.2, 2.0, 1.5), (0.8, 0.2, 0.95, 1.0, 1 / 1.5),
        (0.5, 0.5, 0.1, 0.0, 2.4), (1.0, 1.0, 0.7, 3.0, 1 / 1.33)]


@pytest.mark.parametrize("ax,ay,mu,phi,eta", GEOM)
def test_sample_geometry(orc, ax, ay, mu, phi, eta):
    n = 20000
    wi = _unit(mu, phi, n)
    r = orc.dielectric_sample(wi, ax, ay, eta, seed=11)
    W = np.stack(wi, axis=-1)
    wo, h, lobe = r["wo"], r["h"], r["lobe"]
    np.testing.assert_allclose(np.linalg.norm(wo, axis=1), 1.0, atol=1e-12)
    np.testing.assert_allclose(np.linalg.norm(h, axis=1), 1.0, atol=1e-12)
    ci = np.einsum("ij,ij->i", W, h)
    co = np.einsum("ij,ij->i", wo, h)
    assert np.all(ci > 0)
    # coplanarity of wi, h, wo
    det = np.einsum("ij,ij->i", np.cross(W, h), wo)
    np.testing.assert_allclose(det, 0.0, atol=1e-12)
    R, T = lobe == 0, lobe == 1
    assert np.all(R | T)
    # law of reflection
    np.testing.assert_allclose(co[R], ci[R], atol=1e-12)
    # Snell's law about h, transmitted ray on the far side of the facet
    assert np.all(co[T] < 0)
    si = np.linalg.norm(np.cross(W[T], h[T]), axis=1)
    so = np.linalg.norm(np.cross(wo[T], h[T]), axis=1)
    np.testing.assert_allclose(eta * so, si, atol=1e-12)
    # half vector from the pair: wi + wo (reflection), -(wi + eta wo) (transmission)
    hr = W[R] + wo[R]
    hr /= np.linalg.norm(hr, axis=1)[:, None]
    np.testing.assert_allclose(hr, h[R], atol=1e-9)
    ht = -(W[T] + eta * wo[T])
    ht *= np.sign(ht[:, 2])[:, None] / np.linalg.norm(ht, axis=1)[:, None]
    np.testing.assert_allclose(ht, h[T], atol=1e-9)
    # lobe validity: valid samples on their lobe's side, invalid ones have no density
    valid = r["pdf"] > 0
    assert np.all(wo[R & valid, 2] > 0) and np.all(wo[T & valid, 2] < 0)
    assert np.all(r["weight"][~valid] == 0)
    assert np.all((wo[R & ~valid, 2] <= 0)) and np.all(wo[T & ~valid, 2] >= 0)


@pytest.mark.parametrize("eta", ETAS)
def test_smooth_limit(orc, eta):
    n = 40000
    for mu, phi in ((0.9, 0.3), (0.4, 2.0), (0.15, 4.0)):
        wi = _unit(mu, phi, n)
        r = orc.dielectric_sample(wi, 1e-9, 1e-9, eta, seed=3)
        W = np.stack(wi, axis=-1)
        f = orc.fresnel_dielectric([mu], eta)[0]
        frac = np.mean(r["lobe"] == 0)
        assert abs(frac - f) <= 5 * math.sqrt(max(f * (1 - f), 1e-12) / n) + 1e-12
        R, T = r["lobe"] == 0, r["lobe"] == 1
        np.testing.assert_allclose(r["wo"][R], W[R] * [-1, -1, 1], atol=1e-5)
        if T.any():
            k = 1.0 - (1.0 - mu * mu) / eta ** 2
            snell = np.array([-W[0, 0] / eta, -W[0, 1] / eta, -math.sqrt(k)])
            np.testing.assert_allclose(r["wo"][T], np.broadcast_to(snell, r["wo"][T].shape), atol=1e-5)
        # smooth interface: the weights are all one
        np.testing.assert_allclose(r["weight"], 1.0, atol=1e-5)


# ---------------------------------------------------------------------------
# Densities and weights
# ---------------------------------------------------------------------------

def _sphere_grid(panels, lower, q=4):
    """Composite Gauss-Legendre nodes (panels x q per axis) over one hemisphere
    in (cos theta, phi).  Composite, because the pdf has jumps (where a lobe's
    directions end), which defeat a single high-order rule."""
    x, wq = np.polynomial.legendre.leggauss(q)
    te = np.linspace(0.0, 1.0, panels + 1)
    pe = np.linspace(0.0, 2 * np.pi, panels + 1)
    t = (te[:-1, None] + np.diff(te)[:, None] * (x + 1) / 2).ravel()
    wt = (np.diff(te)[:, None] * wq / 2).ravel()
    p = (pe[:-1, None] + np.diff(pe)[:, None] * (x + 1) / 2).ravel()
    wp = (np.diff(pe)[:, None] * wq / 2).ravel()
    T, P = np.meshgrid(t, p, indexing="ij")
    WT, WP = np.meshgrid(wt, wp, indexing="ij")
    s = np.sqrt(1 - T * T)
    z = -T if lower else T
    d = np.stack([s * np.cos(P), s * np.sin(P), z], axis=-1).reshape(-1, 3)
    return d, (WT * WP).reshape(-1)


NORM = [(0.4, 0.4, 0.6, 0.5, 1.5), (0.3, 0.7, 0.3, 1.2, 1.5), (0.5, 0.5, 0.8, 0.0, 1 / 1.5),
        (0.6, 0.25, 0.25, 2.5, 1.33)]


@pytest.mark.parametrize("ax,ay,mu,phi,eta", NORM)
def test_normalisation_per_lobe(orc, ax, ay, mu, phi, eta):
    n_mc = 1 << 21
    wi = _unit(mu, phi, n_mc)
    r = orc.dielectric_sample(wi, ax, ay, eta, seed=5)
    valid = r["pdf"] > 0
    pR = np.mean(valid & (r["lobe"] == 0))
    pT = np.mean(valid & (r["lobe"] == 1))
    for lower, p in ((False, pR), (True, pT)):
        d, w = _sphere_grid(150, lower)
        m = d.shape[0]
        pdf, _ = orc.dielectric_eval(_unit(mu, phi, m), (d[:, 0], d[:, 1], d[:, 2]), ax, ay, eta)
        integral = float(np.sum(pdf * w))
        sigma = math.sqrt(p * (1 - p) / n_mc)
        assert abs(integral - p) <= 5 * sigma + 2e-5, (lower, integral, p)


@pytest.mark.parametrize("ax,ay,mu,phi,eta", NORM[:3])
def test_chi2_sampled_directions(orc, ax, ay, mu, phi, eta):
    n = 1 << 20
    wi = _unit(mu, phi, n)
    r = orc.dielectric_sample(wi, ax, ay, eta, seed=9)
    valid = r["pdf"] > 0
    wo = r["wo"][valid]
    t_edges = np.linspace(-1.0, 1.0, 25)
    p_edges = np.linspace(0.0, 2 * np.pi, 25)
    counts, _, _ = np.histogram2d(wo[:, 2], np.mod(np.arctan2(wo[:, 1], wo[:, 0]), 2 * np.pi),
                                  bins=[t_edges, p_edges])
    # expected counts: composite Gauss-Legendre inside every bin (6 x 6
    # sub-panels of 4 x 4 nodes), robust to the pdf's jumps
    x, wq = np.polynomial.legendre.leggauss(4)
    sub = 6

    def nodes(edges):
        fine = np.linspace(edges[:-1], edges[1:], sub + 1, axis=1)       # (bins, sub+1)
        lo, wd = fine[:, :-1], np.diff(fine, axis=1)
        pts = (lo[:, :, None] + wd[:, :, None] * (x + 1) / 2).reshape(len(edges) - 1, -1)
        wts = (wd[:, :, None] * wq / 2).reshape(len(edges) - 1, -1)
        return pts, wts

    t, wt = nodes(t_edges)
    p, wp = nodes(p_edges)
    nt, npb, nq = t.shape[0], p.shape[0], t.shape[1]
    T = np.broadcast_to(t[:, None, :, None], (nt, npb, nq, nq))
    P = np.broadcast_to(p[None, :, None, :], (nt, npb, nq, nq))
    W = wt[:, None, :, None] * wp[None, :, None, :]
    s = np.sqrt(1 - T * T)
    d = np.stack([s * np.cos(P), s * np.sin(P), T], axis=-1).reshape(-1, 3)
    m = d.shape[0]
    pdf, _ = orc.dielectric_eval(_unit(mu, phi, m), (d[:, 0], d[:, 1], d[:, 2]), ax, ay, eta)
    expected = (pdf.reshape(nt, npb, nq, nq) * W).sum(axis=(2, 3)) * n
    e, c = expected.ravel(), counts.ravel()
    big = e >= 5
    e = np.append(e[big], e[~big].sum() + n * (1 - valid.mean()) + 1e-300)
    c = np.append(c[big], c[~big].sum() + (~valid).sum())
    scale = c.sum() / e.sum()
    assert abs(scale - 1) < 2e-3
    chi2 = float(np.sum((c - e) ** 2 / e))
    dof = len(e) - 1
    # p > 1e-3 for a chi-square with dof degrees of freedom (Wilson-Hilferty)
    z = ((chi2 / dof) ** (1 / 3) - (1 - 2 / (9 * dof))) / math.sqrt(2 / (9 * dof))
    assert z < 3.1, (chi2, dof)


@pytest.mark.parametrize("ax,ay,mu,phi,eta", GEOM)
def test_weight_closed_form(orc, ax, ay, mu, phi, eta):
    n = 20000
    wi = _unit(mu, phi, n)
    r = orc.dielectric_sample(wi, ax, ay, eta, seed=2)
    valid = r["pdf"] > 0
    W = np.stack(wi, axis=-1)[valid]
    li = _lam(W, ax, ay)
    lo = _lam(r["wo"][valid], ax, ay)
    np.testing.assert_allclose(r["weight"][valid], (1 + li) / (1 + li + lo), rtol=1e-9)
    assert np.all(r["weight"] <= 1.0 + 1e-12)


@pytest.mark.parametrize("ax,ay,mu,phi,eta", GEOM)
def test_bsdf_reciprocity(orc, ax, ay, mu, phi, eta):
    n = 5000
    wi = _unit(mu, phi, n)
    r = orc.dielectric_sample(wi, ax, ay, eta, seed=4)
    valid = r["pdf"] > 0
    W = np.stack(wi, axis=-1)[valid]
    wo = r["wo"][valid]
    lobe = r["lobe"][valid]
    _, f = orc.dielectric_eval(tuple(W.T), tuple(wo.T), ax, ay, eta)
    R, T = lobe == 0, lobe == 1
    # reflection: f(wi, wo) = f(wo, wi)
    _, fr = orc.dielectric_eval(tuple(wo[R].T), tuple(W[R].T), ax, ay, eta)
    np.testing.assert_allclose(f[R], fr, rtol=1e-9)
    # transmission: flip the frame so that wo arrives from above, medium ratio 1/eta
    flip = np.array([1.0, 1.0, -1.0])
    _, ft = orc.dielectric_eval(tuple((wo[T] * flip).T), tuple((W[T] * flip).T), ax, ay, 1.0 / eta)
    np.testing.assert_allclose(f[T], eta * eta * ft, rtol=1e-9)


def test_sampler_pdf_matches_evaluation(orc):
    n = 20000
    wi = _unit(0.5, 1.0, n)
    r = orc.dielectric_sample(wi, 0.2, 0.6, 1.5, seed=8)
    pdf, _ = orc.dielectric_eval(wi, tuple(r["wo"].T), 0.2, 0.6, 1.5)
    v = r["pdf"] > 0
    np.testing.assert_allclose(r["pdf"][v], pdf[v], rtol=1e-9)


def test_uniform_stream_layout(orc):
    seed = 0x0123456789ABCDEF
    u1, u2, u3 = orc.dielectric_uniforms(6, seed, index_base=(1 << 32) + 5)
    for i in range(6):
        k = (1 << 32) + 5 + i
        w = orc.philox4x32_10([k & 0xFFFFFFFF, 0, 5, k >> 32], [seed & 0xFFFFFFFF, seed >> 32])
        assert (u1[i], u2[i], u3[i]) == tuple((int(x) >> 8) * 2.0 ** -24 for x in w[:3])


def test_domain_and_arguments(orc):
    wi = (np.array([0.0, 0.1]), np.array([0.0, 0.0]), np.array([-1.0, 0.99]))
    r = orc.dielectric_sample(wi, np.array([0.3, 0.0]), 0.3, 1.5, seed=1)
    assert np.all(r["lobe"] == -1) and np.all(r["pdf"] == 0) and np.all(r["weight"] == 0)
    with pytest.raises(ValueError):
        orc.dielectric_sample(wi, 0.3, 0.3, 1.0)
    with pytest.raises(ValueError):
        orc.dielectric_sample(wi, 0.3, 0.3, -1.5)
